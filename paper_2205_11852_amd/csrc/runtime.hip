// Error reporting, device contexts, pinned staging and stream-ordered scratch.
#include <cstring>
#include <map>

#include "lc_internal.hpp"

namespace lc {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

lc_status fail(lc_status code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static std::mutex g_ctx_mu;
static std::map<int, DeviceCtx*> g_ctx;

lc_status get_ctx(DeviceCtx** out) {
    int dev = 0;
    LC_TRY_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    auto it = g_ctx.find(dev);
    if (it != g_ctx.end()) {
        *out = it->second;
        return LC_OK;
    }
    auto* c = new DeviceCtx();
    c->device = dev;
    hipDeviceProp_t prop;
    LC_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    c->n_cu = prop.multiProcessorCount;
    c->max_lds_block = prop.sharedMemPerBlock;
    // keep freed stream-ordered memory in the pool between calls
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    LC_TRY_HIP(hipEventCreateWithFlags(&c->pinned_ev, hipEventDisableTiming));
    g_ctx[dev] = c;
    *out = c;
    return LC_OK;
}

size_t Stager::push(const void* src, size_t bytes) {
    size_t off = (host_.size() + 255) & ~size_t(255);
    host_.resize(off + bytes);
    if (bytes) std::memcpy(host_.data() + off, src, bytes);
    return off;
}

lc_status Stager::commit(hipStream_t s, void** dev_base) {
    size_t n = host_.size() ? host_.size() : 1;
    std::lock_guard<std::mutex> lk(ctx_->mu);
    if (ctx_->pinned_pending) {
        // the previous copy out of the pinned block must have finished
        LC_TRY_HIP(hipEventSynchronize(ctx_->pinned_ev));
        ctx_->pinned_pending = false;
    }
    if (ctx_->pinned_size < n) {
        if (ctx_->pinned) LC_TRY_HIP(hipHostFree(ctx_->pinned));
        ctx_->pinned = nullptr;
        size_t sz = 1 << 16;
        while (sz < n) sz <<= 1;
        if (hipHostMalloc(&ctx_->pinned, sz, hipHostMallocDefault) != hipSuccess) {
            ctx_->pinned = nullptr;
            ctx_->pinned_size = 0;
            return fail(LC_ERR_NOMEM, "pinned staging allocation of %zu bytes failed", sz);
        }
        ctx_->pinned_size = sz;
    }
    if (!host_.empty()) std::memcpy(ctx_->pinned, host_.data(), host_.size());
    void* d = nullptr;
    LC_TRY(dev_alloc(&d, n, s));
    if (!host_.empty())
        LC_TRY_HIP(hipMemcpyAsync(d, ctx_->pinned, host_.size(), hipMemcpyHostToDevice, s));
    LC_TRY_HIP(hipEventRecord(ctx_->pinned_ev, s));
    ctx_->pinned_pending = true;
    *dev_base = d;
    return LC_OK;
}

lc_status dev_alloc(void** p, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMallocAsync(p, bytes, s);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? LC_ERR_NOMEM : LC_ERR_HIP,
                    "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    return LC_OK;
}

void dev_free(void* p, hipStream_t s) {
    if (p) (void)hipFreeAsync(p, s);
}

}  // namespace lc

extern "C" const char* lc_last_error(void) { return lc::g_err.c_str(); }

extern "C" void lc_release_caches(void) {
    lc::DeviceCtx* c = nullptr;
    if (lc::get_ctx(&c) != LC_OK) return;
    lc::release_graphs();
    lc::release_tuning();
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->pinned_pending) (void)hipEventSynchronize(c->pinned_ev);
    c->pinned_pending = false;
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_size = 0;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) {
        (void)hipDeviceSynchronize();
        (void)hipMemPoolTrimTo(pool, 0);
    }
}
