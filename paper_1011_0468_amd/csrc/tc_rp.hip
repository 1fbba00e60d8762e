// Random-projection trace estimator (section 5.1).  The paper projects the
// adjacency columns with a Gaussian matrix R and shows E[Y] = k tr(A^3) for
// Y = sum_l r_l^T A^3 r_l.  Here each r_l is a Rademacher vector x_l (the same
// mean, E[x_i x_j] = delta_ij) so that q_l = x_l^T A^3 x_l = (A x_l)^T A (A x_l)
// is an exact integer.  Vectors are processed 64 at a time: one 64-bit hash
// word per vertex holds the 64 signs of a chunk, and lane b of a wave owns
// vector b of the chunk.
//
//   word[i] = mix64(mix64(c << 32 | i) ^ salt)       (computed where it is used)
//   rp_spmm : Y[i][b] = sum_{j in N(i)} x_b[j] = deg i - 2 #{j in N(i) : bit b of word[j]}
//             (per batch of 64 entries: a 64 x 64 bit transpose, then one masked
//             popcount per lane and run of one row)
//   rp_dot  : q[b]    = sum over CSR entries (i, j) of Y[i][b] * Y[j][b]
//                     = 2 * sum over the entries with j > i
//
// Both sweeps are edge-parallel: wave w owns CSR entries [w L, (w+1) L), so a
// hub row is split over many waves.  rp_dot is a plain sum over entries.  In
// rp_spmm a row that lies entirely inside one wave's range is stored
// directly; the partial rows at range boundaries are accumulated atomically
// into rows that rp_clear_ends zeroes first (the count is additive over any
// split of the row).
#include "tc_internal.h"
#include "tc_device.h"

#include <vector>

namespace tc {

namespace {

constexpr int kRpRange = 4096;  // CSR entries per wave
constexpr int kRpUnroll = 8;    // entries whose loads are issued together

// The 64 signs of vertex i in chunk c (bit b set: x_{64c+b}[i] = -1).
__device__ __forceinline__ uint64_t sign_word(uint64_t chunk, int32_t i, uint64_t salt) {
    return mix64(mix64((chunk << 32) | (uint64_t)(uint32_t)i) ^ salt);
}

__device__ __forceinline__ void rp_flush(int32_t i, int32_t cnt, int32_t ones, int64_t e0, int64_t e1,
                                         const int32_t* __restrict__ row_ptr, int32_t* __restrict__ Y, int lane) {
    const int32_t val = cnt - 2 * ones;
    if ((int64_t)row_ptr[i] >= e0 && (int64_t)row_ptr[i + 1] <= e1) Y[(int64_t)i * 64 + lane] = val;
    else atomicAdd(&Y[(int64_t)i * 64 + lane], val);
}

// Lane exchange with lane ^ J of a 32-bit value (ds_swizzle inside each half
// of the wave, a permute across the halves).
template <int J>
__device__ __forceinline__ uint32_t rp_xor(uint32_t v) {
    if constexpr (J < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1F);
    else return (uint32_t)__shfl_xor((int)v, J, 64);
}

// Level J < 32 of the 64 x 64 bit transpose on one 32-bit half (m: the bits
// whose index has bit J clear).  Bit c of lane l moves to bit c ^ J of lane
// l ^ J when bit J of l and bit J of c differ, and stays otherwise.
template <int J>
__device__ __forceinline__ uint32_t transpose_level(uint32_t x, uint32_t m, bool hi_lane) {
    const uint32_t o = rp_xor<J>(x);
    return hi_lane ? ((x & ~m) | ((o >> J) & m)) : ((x & m) | ((o << J) & ~m));
}

// Transposes the 64 x 64 bit matrix whose row l is lane l's word (lo, hi):
// afterwards bit k of lane b's word is bit b of lane k's word.  Each level J
// exchanges the elements whose row and column differ in bit J; the levels
// act on different bits of (row xor column), so together they swap every
// element with its mirror.  Whole wave.
__device__ __forceinline__ void transpose64(uint32_t& lo, uint32_t& hi, int lane) {
    {
        const bool h = (lane & 32) != 0;
        const uint32_t got = rp_xor<32>(h ? lo : hi);  // the half the partner keeps below / above
        if (h) lo = got; else hi = got;
    }
    lo = transpose_level<16>(lo, 0x0000FFFFu, (lane & 16) != 0);
    hi = transpose_level<16>(hi, 0x0000FFFFu, (lane & 16) != 0);
    lo = transpose_level<8>(lo, 0x00FF00FFu, (lane & 8) != 0);
    hi = transpose_level<8>(hi, 0x00FF00FFu, (lane & 8) != 0);
    lo = transpose_level<4>(lo, 0x0F0F0F0Fu, (lane & 4) != 0);
    hi = transpose_level<4>(hi, 0x0F0F0F0Fu, (lane & 4) != 0);
    lo = transpose_level<2>(lo, 0x33333333u, (lane & 2) != 0);
    hi = transpose_level<2>(hi, 0x33333333u, (lane & 2) != 0);
    lo = transpose_level<1>(lo, 0x55555555u, (lane & 1) != 0);
    hi = transpose_level<1>(hi, 0x55555555u, (lane & 1) != 0);
}

// Y = A X over the wave's entry range, 64 entries per batch: lane k loads
// entry k and computes its neighbour's sign word (hashing is cheaper than a
// random 8-byte gather per entry), the 64 words are transposed so that lane b
// holds bit b of every entry's word, and each run of entries of one row adds
// its length to cnt and its masked popcount to ones (lane b: the entries
// whose sign b is negative).  A row is written when the next one starts.
__global__ void __launch_bounds__(256) k_rp_spmm(int64_t E2, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                  uint64_t chunk, uint64_t salt, int32_t* __restrict__ Y) {
    const int lane = __lane_id();
    const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t e0 = w * kRpRange;
    if (e0 >= E2) return;
    const int64_t e1 = e0 + kRpRange < E2 ? e0 + kRpRange : E2;
    int32_t cur = __builtin_amdgcn_readfirstlane(src[e0]);
    int32_t cnt = 0, ones = 0;
    for (int64_t eb = e0; eb < e1; eb += 64) {
        const int64_t el = eb + lane;
        const bool valid = el < e1;
        const int32_t vi = valid ? src[el] : -1;
        const int32_t vj = valid ? col[el] : 0;
        const uint64_t wv = valid ? sign_word(chunk, vj, salt) : 0ull;
        uint32_t lo = (uint32_t)wv, hi = (uint32_t)(wv >> 32);
        transpose64(lo, hi, lane);
        int32_t prev = __shfl_up(vi, 1, 64);
        if (lane == 0) prev = cur;
        const uint64_t V = ballot64(valid);               // a prefix of the lanes
        const uint64_t S = ballot64(valid && vi != prev);  // entries that start a row
        uint64_t rest = V;
        while (rest) {  // wave-uniform: one pass per run of one row
            const int k0 = __builtin_ctzll(rest);
            if ((S >> k0) & 1ull) {
                rp_flush(cur, cnt, ones, e0, e1, row_ptr, Y, lane);
                cur = __builtin_amdgcn_readlane(vi, k0);
                cnt = 0;
                ones = 0;
            }
            const uint64_t after = S & (~1ull << k0);  // row starts past k0
            const uint64_t run = after ? rest & ((1ull << __builtin_ctzll(after)) - 1ull) : rest;
            cnt += (int32_t)__popcll(run);
            ones += (int32_t)(__builtin_popcount(lo & (uint32_t)run) + __builtin_popcount(hi & (uint32_t)(run >> 32)));
            rest &= ~run;
        }
    }
    rp_flush(cur, cnt, ones, e0, e1, row_ptr, Y, lane);
}

// Clears the rows of Y that k_rp_spmm accumulates atomically: a row split
// between two wave ranges is the last row of one and the first of the next,
// so clearing the first and last row of every range covers them (the other
// rows are stored whole, and rows without entries are never read).
__global__ void __launch_bounds__(256) k_rp_clear_ends(int64_t E2, const int32_t* __restrict__ src,
                                                        int32_t* __restrict__ Y) {
    const int lane = __lane_id();
    const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t e0 = w * kRpRange;
    if (e0 >= E2) return;
    const int64_t e1 = e0 + kRpRange < E2 ? e0 + kRpRange : E2;
    Y[(int64_t)src[e0] * 64 + lane] = 0;
    Y[(int64_t)src[e1 - 1] * 64 + lane] = 0;
}

// q[b] = sum over CSR entries (i, j) of Y[i][b] Y[j][b] = 2 * the sum over the
// entries with j > i (A is symmetric without loops), so only those entries
// gather the 256-byte row Y[j]; the entry indices are wave-uniform and kept in
// scalar registers (read from lanes of one coalesced load), so a skipped
// entry issues no load.
__global__ void __launch_bounds__(256) k_rp_dot(int64_t E2, const int32_t* __restrict__ src,
                                                 const int32_t* __restrict__ col, const int32_t* __restrict__ Y,
                                                 int64_t* __restrict__ q) {
    const int lane = __lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * 4 + wv;
    const int64_t e0 = w * kRpRange;
    int64_t acc = 0;
    if (e0 < E2) {
        const int64_t e1 = e0 + kRpRange < E2 ? e0 + kRpRange : E2;
        int32_t cur = -1, ycur = 0;
        for (int64_t eb = e0; eb < e1; eb += 64) {
            // 64 entries per coalesced load; entry k of the batch is read from lane k
            const int64_t el = eb + lane;
            const int32_t vi = el < e1 ? src[el] : -1;
            const int32_t vj = el < e1 ? col[el] : -1;
            for (int k0 = 0; k0 < 64; k0 += kRpUnroll) {
                int32_t ii[kRpUnroll], jj[kRpUnroll], yj[kRpUnroll];
#pragma unroll
                for (int k = 0; k < kRpUnroll; ++k) {
                    ii[k] = __builtin_amdgcn_readlane(vi, k0 + k);
                    jj[k] = __builtin_amdgcn_readlane(vj, k0 + k);
                }
#pragma unroll
                for (int k = 0; k < kRpUnroll; ++k) yj[k] = jj[k] > ii[k] ? Y[(int64_t)jj[k] * 64 + lane] : 0;
#pragma unroll
                for (int k = 0; k < kRpUnroll; ++k) {
                    if (jj[k] <= ii[k]) continue;  // lower entry, or past the range end (-1, -1)
                    if (ii[k] != cur) {
                        cur = ii[k];
                        ycur = Y[(int64_t)cur * 64 + lane];
                    }
                    acc += (int64_t)ycur * (int64_t)yj[k];
                }
            }
        }
    }
    __shared__ int64_t red[4][64];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0) {
        const int64_t s = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
        if (s) atomicAdd((unsigned long long*)&q[lane], (unsigned long long)(2 * s));
    }
}

// Half the sum over CSR entries (i, j) of deg_i * deg_j, in double (a bound
// only): the entries with j > i, whose mirrors give the same sum, so only
// they gather deg_j.  One partial per block, summed on the host.
__global__ void __launch_bounds__(256) k_rp_bound(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ deg, int64_t E2,
                                                   double* __restrict__ part) {
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E2; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = src[e], j = col[e];
        if (j > i) s += (double)deg[i] * (double)deg[j];
    }
    s = wave_sum(s);
    __shared__ double red[4];
    if (__lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

}  // namespace

void rp_trace(const tc_graph_s* g, int32_t k, uint64_t seed, hipStream_t s, int64_t* q_host) {
    PhaseScope ph("rp");
    const int64_t n = g->n, E2 = 2 * g->m;
    for (int32_t l = 0; l < k; ++l) q_host[l] = 0;
    if (n == 0 || E2 == 0) return;
    {
        // |q_l| <= sum over entries (i, j) of |Y_il| |Y_jl| <= sum of deg_i deg_j; every q_l and their sum
        // stay exact while k times that is below 2^62 (margin for the double rounding)
        unsigned blocks = ceil_div(E2, 256);
        if (blocks > 1024) blocks = 1024;
        DevBuf<double> part(blocks, s);
        TC_LAUNCH("rp_bound", k_rp_bound, dim3(blocks), dim3(256), 0, s, (const int32_t*)g->src,
                  (const int32_t*)g->col, (const int32_t*)g->deg, E2, part.get());
        std::vector<double> hpart(blocks);
        check_hip(hipMemcpyAsync(hpart.data(), part.get(), sizeof(double) * blocks, hipMemcpyDeviceToHost, s),
                  "bound");
        check_hip(hipStreamSynchronize(s), "sync");
        double hb = 0.0;
        for (double v : hpart) hb += v;
        hb *= 2.0;
        if (hb * (double)k >= 4.611686018427387904e18)
            fail(TC_ERR_OVERFLOW, "k * sum deg_i deg_j reaches 2^62: q could overflow int64");
    }
    const uint64_t salt = [&] {
        uint64_t z = seed ^ 0x52505F5452414345ull;  // "RP_TRACE"
        z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull; z ^= z >> 27; z *= 0x94D049BB133111EBull; z ^= z >> 31;
        return z;
    }();
    DevBuf<int32_t> Y((size_t)n * 64, s);
    DevBuf<int64_t> qd(64, s);
    const int32_t nchunks = (k + 63) / 64;
    const int64_t waves = (E2 + kRpRange - 1) / kRpRange;
    const unsigned wblocks = (unsigned)((waves + 3) / 4);
    for (int32_t c = 0; c < nchunks; ++c) {
        fill_i64(qd.get(), 0, 64, s);
        TC_LAUNCH("rp_clear", k_rp_clear_ends, dim3(wblocks), dim3(256), 0, s, E2, (const int32_t*)g->src, Y.get());
        TC_LAUNCH("rp_spmm", k_rp_spmm, dim3(wblocks), dim3(256), 0, s, E2, (const int32_t*)g->row_ptr,
                  (const int32_t*)g->src, (const int32_t*)g->col, (uint64_t)c, salt, Y.get());
        TC_LAUNCH("rp_dot", k_rp_dot, dim3(wblocks), dim3(256), 0, s, E2, (const int32_t*)g->src,
                  (const int32_t*)g->col, (const int32_t*)Y.get(), qd.get());
        int64_t hq[64];
        check_hip(hipMemcpyAsync(hq, qd.get(), sizeof(hq), hipMemcpyDeviceToHost, s), "q");
        check_hip(hipStreamSynchronize(s), "sync");
        for (int b = 0; b < 64 && c * 64 + b < k; ++b) q_host[c * 64 + b] = hq[b];
    }
}

}  // namespace tc
