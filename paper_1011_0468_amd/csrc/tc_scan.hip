// Device-wide exclusive scan (reduce-then-scan) and fill kernels.
#include "tc_internal.h"
#include "tc_device.h"

namespace tc {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int32_t* __restrict__ in, int64_t N,
                                                               int32_t* __restrict__ bsum) {
    __shared__ int32_t tmp[kScanThreads / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;  // coalesced
        if (idx < N) acc += in[idx];
    }
    int32_t total;
    block_exclusive_sum<kScanThreads>(acc, tmp, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Each thread owns kScanItems consecutive items; `bsum` (may be null) holds the
// exclusive block offsets with the grand total at bsum[gridDim.x].
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const int32_t* in, int32_t* out, int64_t N,
                                                              const int32_t* __restrict__ bsum) {
    __shared__ int32_t tmp[kScanThreads / 64 + 1];
    __shared__ int32_t stage[kScanTile + kScanTile / 16];  // padded: index i -> i + i/16
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // coalesced load into LDS
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;
        const int j = i * kScanThreads + threadIdx.x;
        stage[j + (j >> 4)] = idx < N ? in[idx] : 0;
    }
    __syncthreads();
    int32_t v[kScanItems];
    int32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int j = threadIdx.x * kScanItems + i;
        v[i] = stage[j + (j >> 4)];
        acc += v[i];
    }
    int32_t total;
    int32_t pre = block_exclusive_sum<kScanThreads>(acc, tmp, &total);
    const int32_t off = bsum ? bsum[blockIdx.x] : 0;
    pre += off;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int j = threadIdx.x * kScanItems + i;
        stage[j + (j >> 4)] = pre;
        pre += v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;
        const int j = i * kScanThreads + threadIdx.x;
        if (idx < N) out[idx] = stage[j + (j >> 4)];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[N] = bsum ? bsum[gridDim.x] : total;
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
void fill_impl(T* p, T v, int64_t N, hipStream_t s) {
    if (N <= 0) return;
    unsigned blocks = ceil_div(N, 256);
    if (blocks > 8192) blocks = 8192;
    TC_LAUNCH("fill", k_fill<T>, dim3(blocks), dim3(256), 0, s, p, v, N);
}

}  // namespace

void scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t N, hipStream_t s) {
    if (N <= kScanTile) {
        TC_LAUNCH("scan_apply", k_scan_apply, dim3(1), dim3(kScanThreads), 0, s, in, out, N,
                  (const int32_t*)nullptr);
        return;
    }
    const int64_t nb = (N + kScanTile - 1) / kScanTile;
    DevBuf<int32_t> bs(nb + 1, s);
    TC_LAUNCH("scan_reduce", k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, N, bs.get());
    scan_exclusive_i32(bs.get(), bs.get(), nb, s);
    TC_LAUNCH("scan_apply", k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, N,
              (const int32_t*)bs.get());
}

int64_t scan_scratch_bytes(int64_t N) {
    if (N <= kScanTile) return 0;
    const int64_t nb = (N + kScanTile - 1) / kScanTile;
    return region_bytes(4 * (nb + 1)) + scan_scratch_bytes(nb);
}

void fill_i32(int32_t* p, int32_t v, int64_t N, hipStream_t s) { fill_impl<int32_t>(p, v, N, s); }
void fill_i64(int64_t* p, int64_t v, int64_t N, hipStream_t s) { fill_impl<int64_t>(p, v, N, s); }
void fill_u8(uint8_t* p, uint8_t v, int64_t N, hipStream_t s) { fill_impl<uint8_t>(p, v, N, s); }

}  // namespace tc
