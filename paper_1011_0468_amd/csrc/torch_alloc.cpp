// Device allocation through PyTorch's caching allocator, for tc_set_allocator:
// the library's buffers then come from the same pool as the caller's tensors
// (no second cache of device memory beside torch's).  Host code only.
#include <c10/hip/HIPCachingAllocator.h>

#include <cstddef>

extern "C" void* tc_torch_alloc(size_t bytes, void* stream, void* /*ctx*/) {
    try {
        return c10::hip::HIPCachingAllocator::raw_alloc_with_stream(bytes, static_cast<hipStream_t>(stream));
    } catch (...) {
        return nullptr;  // the library reports TC_ERR_OOM
    }
}

extern "C" void tc_torch_free(void* ptr, void* /*stream*/, void* /*ctx*/) {
    try {
        c10::hip::HIPCachingAllocator::raw_delete(ptr);
    } catch (...) {
    }
}
