// Allocation-free variant of the single-seed estimate, for callers that may not
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Every buffer of the count comes from one
// fixed device array, `scratch`, reserved with the code object: the call makes
// no hipMalloc, hipFree or other allocating call, and counts exactly what
// tc_estimate counts for the same (graph, p, seed, params).
#include "tc_internal.h"

#include <mutex>
#include <string>
#include <vector>

namespace tc {

// Bytes of the device scratch array (each GPU the library runs on holds one
// copy until the process ends).
constexpr int64_t kScratchBytes = (int64_t)64 << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

// Device address of each GPU's copy of `scratch`, resolved once per device
// with that device current.  In host code the array's name is only a host-side
// stand-in, so every use below goes through these addresses.
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};
// One call at a time per device: every call shares that device's array.
std::mutex g_device_mu[kMaxDevices];

unsigned char* scratch_for(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (!p) fail(TC_ERR_DEVICE, "scratch symbol address is NULL");
        g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
    }
    return g_scratch_ptr[dev];
}

// Stack of allocations inside the scratch array; anything that does not fit
// is an error (never a fall-back to the installed allocator).
class ScratchStack : public AllocRegion {
public:
    ScratchStack(unsigned char* base, int64_t size) : base_(base), size_(size) { strict = true; }
    void* try_alloc(size_t bytes) override {
        const int64_t b = region_bytes((int64_t)bytes);
        if (top_ + b > size_) return nullptr;
        void* p = base_ + top_;
        blocks_.push_back({top_, false});
        top_ += b;
        return p;
    }
    bool try_free(void* p) override {
        unsigned char* c = static_cast<unsigned char*>(p);
        if (c < base_ || c >= base_ + size_) return false;
        const int64_t off = c - base_;
        for (auto it = blocks_.rbegin(); it != blocks_.rend(); ++it)
            if (it->off == off && !it->freed) {
                it->freed = true;
                break;
            }
        while (!blocks_.empty() && blocks_.back().freed) {
            top_ = blocks_.back().off;
            blocks_.pop_back();
        }
        return true;
    }

private:
    struct Block {
        int64_t off;
        bool freed;
    };
    unsigned char* base_;
    int64_t size_;
    int64_t top_ = 0;
    std::vector<Block> blocks_;
};

struct RegionGuard {
    AllocRegion* prev;
    explicit RegionGuard(AllocRegion* r) : prev(set_thread_region(r)) {}
    ~RegionGuard() { set_thread_region(prev); }
};

}  // namespace

}  // namespace tc

using namespace tc;

extern "C" tc_status tc_estimate_noalloc(tc_graph g, double p, uint64_t seed, const tc_params* prm, void* stream,
                                         tc_counts* out, double* est) {
    try {
        set_last_error("");
        if (!g || !out) fail(TC_ERR_INVALID, "graph or output is NULL");
        if (!p_valid(p)) fail(TC_ERR_INVALID, "p must be finite and in (0, 1]");
        const int sampled = p < 1.0 ? 1 : 0;
        const CountConfig cfg = config_from(prm, g, sampled, p);
        const int64_t need = count_bytes(g->n, g->m, g->max_deg, sampled, cfg);
        if (need > kScratchBytes)
            fail(TC_ERR_BUDGET, "the count needs " + std::to_string(need) + " bytes of scratch; the limit is " +
                                    std::to_string(kScratchBytes));
        int dev = 0;
        check_hip(hipGetDevice(&dev), "get device");
        if (dev < 0 || dev >= kMaxDevices) fail(TC_ERR_DEVICE, "device index out of range");
        hipStream_t s = (hipStream_t)stream;
        std::lock_guard<std::mutex> lk(g_device_mu[dev]);
        unsigned char* base = scratch_for(dev);
        ScratchStack region(base, kScratchBytes);
        RegionGuard guard(&region);
        NoProfileScope quiet;  // profiling events would be created on demand: none in this call
        tc_counts r;
        try {
            count_core(g, sampled, keep_threshold(p), sample_salt(seed), cfg, s, &r);
        } catch (...) {
            (void)hipStreamSynchronize(s);  // nothing of this call may still use the array
            throw;
        }
        *out = r;
        if (est) *est = rescale(r.triangles, p);
        profile_collect();
        return TC_OK;
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return TC_ERR_DEVICE;
    } catch (...) {
        set_last_error("unknown error");
        return TC_ERR_DEVICE;
    }
}
