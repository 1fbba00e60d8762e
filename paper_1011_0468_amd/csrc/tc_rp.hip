// Random-projection trace estimator (section 5.1).  The paper projects the
// adjacency columns with a Gaussian matrix R and shows E[Y] = k tr(A^3) for
// Y = sum_l r_l^T A^3 r_l.  Here each r_l is a Rademacher vector x_l (the same
// mean, E[x_i x_j] = delta_ij) so that q_l = x_l^T A^3 x_l = (A x_l)^T A (A x_l)
// is an exact integer.  Vectors are processed 64 at a time: one 64-bit hash
// word per vertex holds the 64 signs of a chunk.
//
//   rp_bits : word[i] = mix64(mix64(c << 32 | i) ^ salt)          (n words)
//   rp_spmm : Y[i][b] = sum_{j in N(i)} x_b[j] = deg i - 2 #{j : bit b set}
//   rp_dot  : q[b]  += Y[i][b] * sum_{j in N(i)} Y[j][b]
#include "tc_internal.h"
#include "tc_device.h"

namespace tc {

namespace {

__global__ void k_rp_bits(int64_t n, uint64_t chunk, uint64_t salt, uint64_t* __restrict__ words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        words[i] = mix64(mix64((chunk << 32) | (uint64_t)i) ^ salt);
}

// one wave per vertex (grid-stride); lane b owns sign bit b
__global__ void __launch_bounds__(256) k_rp_spmm(int64_t n, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col, const uint64_t* __restrict__ words,
                                                  int32_t* __restrict__ Y) {
    __shared__ uint64_t stage[4][64];
    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < n; i += nw) {
        const int32_t b0 = row_ptr[i], b1 = row_ptr[i + 1];
        int32_t ones = 0;
        for (int32_t e0 = b0; e0 < b1; e0 += 64) {
            const int32_t e = e0 + lane;
            stage[w][lane] = e < b1 ? words[col[e]] : 0ull;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const int cnt = min(64, b1 - e0);
            for (int t = 0; t < cnt; ++t) ones += (int32_t)((stage[w][t] >> lane) & 1ull);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        Y[i * 64 + lane] = (b1 - b0) - 2 * ones;
    }
}

__global__ void __launch_bounds__(256) k_rp_dot(int64_t n, const int32_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col, const int32_t* __restrict__ Y,
                                                 int64_t* __restrict__ q) {
    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    const int64_t nw = (int64_t)gridDim.x * 4;
    int64_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < n; i += nw) {
        const int32_t b0 = row_ptr[i], b1 = row_ptr[i + 1];
        int64_t z = 0;
        for (int32_t e = b0; e < b1; ++e) z += Y[(int64_t)col[e] * 64 + lane];
        acc += (int64_t)Y[i * 64 + lane] * z;
    }
    __shared__ int64_t red[4][64];
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
        const int64_t s = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
        if (s) atomicAdd((unsigned long long*)&q[lane], (unsigned long long)s);
    }
}

// sum over directed edges (i, j) of deg_i * deg_j, in double (a bound only)
__global__ void k_rp_bound(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ deg, int64_t E2, double* __restrict__ out) {
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E2; e += (int64_t)gridDim.x * blockDim.x)
        s += (double)deg[src[e]] * (double)deg[col[e]];
    s = wave_sum(s);
    if (__lane_id() == 0) atomicAdd(out, s);
}

}  // namespace

void rp_trace(const tc_graph_s* g, int32_t k, uint64_t seed, hipStream_t s, int64_t* q_host) {
    const int64_t n = g->n, E2 = 2 * g->m;
    for (int32_t l = 0; l < k; ++l) q_host[l] = 0;
    if (n == 0 || E2 == 0) return;
    {
        DevBuf<double> bound(1, s);
        fill_i64(reinterpret_cast<int64_t*>(bound.get()), 0, 1, s);  // +0.0
        unsigned blocks = ceil_div(E2, 256);
        if (blocks > 8192) blocks = 8192;
        TC_LAUNCH("rp_bound", k_rp_bound, dim3(blocks), dim3(256), 0, s, (const int32_t*)g->src,
                  (const int32_t*)g->col, (const int32_t*)g->deg, E2, bound.get());
        double hb = 0.0;
        check_hip(hipMemcpyAsync(&hb, bound.get(), sizeof(double), hipMemcpyDeviceToHost, s), "bound");
        check_hip(hipStreamSynchronize(s), "sync");
        // |q_l| <= sum_(i,j) deg_i deg_j; keep k times that below 2^62 (margin for the double rounding)
        if (hb * (double)k >= 4.611686018427387904e18)
            fail(TC_ERR_OVERFLOW, "k * sum deg_i deg_j reaches 2^62: q could overflow int64");
    }
    const uint64_t salt = [&] {
        uint64_t z = seed ^ 0x52505F5452414345ull;  // "RP_TRACE"
        z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull; z ^= z >> 27; z *= 0x94D049BB133111EBull; z ^= z >> 31;
        return z;
    }();
    DevBuf<uint64_t> words(n, s);
    DevBuf<int32_t> Y((size_t)n * 64, s);
    DevBuf<int64_t> qd(64, s);
    const int32_t nchunks = (k + 63) / 64;
    for (int32_t c = 0; c < nchunks; ++c) {
        fill_i64(qd.get(), 0, 64, s);
        unsigned blocks = ceil_div(n, 256);
        if (blocks > 65536) blocks = 65536;
        TC_LAUNCH("rp_bits", k_rp_bits, dim3(blocks), dim3(256), 0, s, n, (uint64_t)c, salt, words.get());
        unsigned wblocks = ceil_div(n, 4);
        if (wblocks > 65536) wblocks = 65536;
        TC_LAUNCH("rp_spmm", k_rp_spmm, dim3(wblocks), dim3(256), 0, s, n, (const int32_t*)g->row_ptr,
                  (const int32_t*)g->col, (const uint64_t*)words.get(), Y.get());
        TC_LAUNCH("rp_dot", k_rp_dot, dim3(wblocks), dim3(256), 0, s, n, (const int32_t*)g->row_ptr,
                  (const int32_t*)g->col, (const int32_t*)Y.get(), qd.get());
        int64_t hq[64];
        check_hip(hipMemcpyAsync(hq, qd.get(), sizeof(hq), hipMemcpyDeviceToHost, s), "q");
        check_hip(hipStreamSynchronize(s), "sync");
        for (int b = 0; b < 64 && c * 64 + b < k; ++b) q_host[c * 64 + b] = hq[b];
    }
}

}  // namespace tc
