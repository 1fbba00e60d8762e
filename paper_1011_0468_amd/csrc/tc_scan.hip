// Device-wide exclusive scan (reduce-then-scan) and fill kernels.
#include "tc_internal.h"
#include "tc_device.h"

namespace tc {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// Up to kScanBatch arrays of one length scanned by the same launches:
// blockIdx.y selects the array; its block sums sit at bsum + y * bstride.
constexpr int kScanBatch = 4;
struct ScanArrays {
    const int32_t* in[kScanBatch];
    int32_t* out[kScanBatch];
};

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(ScanArrays a, int64_t N, int32_t* __restrict__ bsum_all,
                                                               int64_t bstride) {
    const int32_t* __restrict__ in = a.in[blockIdx.y];
    int32_t* __restrict__ bsum = bsum_all + blockIdx.y * bstride;
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

// Each thread owns kScanItems consecutive items; the block sums (null: a
// single block) hold the exclusive block offsets with the grand total at
// [gridDim.x].  in and out may be the same array.
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(ScanArrays a, int64_t N,
                                                              const int32_t* __restrict__ bsum_all, int64_t bstride) {
    const int32_t* in = a.in[blockIdx.y];
    int32_t* out = a.out[blockIdx.y];
    const int32_t* __restrict__ bsum = bsum_all ? bsum_all + blockIdx.y * bstride : nullptr;
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

static void scan_batch(ScanArrays a, int K, int64_t N, hipStream_t s) {
    if (N <= kScanTile) {
        TC_LAUNCH("scan_apply", k_scan_apply, dim3(1, K), dim3(kScanThreads), 0, s, a, N, (const int32_t*)nullptr,
                  (int64_t)0);
        return;
    }
    const int64_t nb = (N + kScanTile - 1) / kScanTile;
    DevBuf<int32_t> bs(K * (nb + 1), s);
    TC_LAUNCH("scan_reduce", k_scan_reduce, dim3((unsigned)nb, K), dim3(kScanThreads), 0, s, a, N, bs.get(), nb + 1);
    ScanArrays b{};
    for (int k = 0; k < K; ++k) b.in[k] = b.out[k] = bs.get() + k * (nb + 1);
    scan_batch(b, K, nb, s);
    TC_LAUNCH("scan_apply", k_scan_apply, dim3((unsigned)nb, K), dim3(kScanThreads), 0, s, a, N,
              (const int32_t*)bs.get(), nb + 1);
}

static int64_t batch_scratch_bytes(int K, int64_t N) {
    if (N <= kScanTile) return 0;
    const int64_t nb = (N + kScanTile - 1) / kScanTile;
    return region_bytes(4 * K * (nb + 1)) + batch_scratch_bytes(K, nb);
}

void scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t N, hipStream_t s) {
    ScanArrays a{};
    a.in[0] = in;
    a.out[0] = out;
    scan_batch(a, 1, N, s);
}

void scan_exclusive_i32_x4(const int32_t* const in[4], int32_t* const out[4], int64_t N, hipStream_t s) {
    static_assert(kScanBatch == 4, "four arrays per batch");
    ScanArrays a{};
    for (int k = 0; k < 4; ++k) {
        a.in[k] = in[k];
        a.out[k] = out[k];
    }
    scan_batch(a, 4, N, s);
}

int64_t scan_scratch_bytes(int64_t N) { return batch_scratch_bytes(1, N); }
int64_t scan_x4_scratch_bytes(int64_t N) { return batch_scratch_bytes(4, N); }

void fill_i32(int32_t* p, int32_t v, int64_t N, hipStream_t s) { fill_impl<int32_t>(p, v, N, s); }
void fill_i64(int64_t* p, int64_t v, int64_t N, hipStream_t s) { fill_impl<int64_t>(p, v, N, s); }
void fill_u8(uint8_t* p, uint8_t v, int64_t N, hipStream_t s) { fill_impl<uint8_t>(p, v, N, s); }

}  // namespace tc
