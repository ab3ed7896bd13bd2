// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "lc.h"

namespace lc {

// Points per catalogue stay below 2^28, so that a point's index within its
// catalogue times 12 bytes is a 32-bit byte offset: the pair kernel gathers
// points by such offsets, and the midpoint line of sight keeps them in a
// 32-bit queue slot.
constexpr int64_t kMaxCatalogue = int64_t(1) << 28;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();
lc_status fail(lc_status code, const char* fmt, ...);

#define LC_TRY_HIP(call)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::lc::fail(LC_ERR_HIP, "%s failed: %s (%s:%d)", #call,                 \
                              hipGetErrorString(e_), __FILE__, __LINE__);                 \
    } while (0)

#define LC_TRY(expr)                                                                      \
    do {                                                                                  \
        lc_status s_ = (expr);                                                            \
        if (s_ != LC_OK) return s_;                                                       \
    } while (0)

// ---------------------------------------------------------------------------
// per-device context
// ---------------------------------------------------------------------------
struct DeviceCtx {
    int device = -1;
    int n_cu = 0;
    size_t max_lds_block = 65536;
    std::mutex mu;
    // pinned staging for small host->device parameter copies; guarded by an
    // event so the host never overwrites bytes a pending copy still reads
    void* pinned = nullptr;
    size_t pinned_size = 0;
    hipEvent_t pinned_ev = nullptr;
    bool pinned_pending = false;
};

// Context of the current device (created on first use).
lc_status get_ctx(DeviceCtx** out);

// Stages host arrays into one pinned block and copies them to a
// stream-ordered device allocation with a single hipMemcpyAsync.
class Stager {
  public:
    explicit Stager(DeviceCtx* c) : ctx_(c) {}
    // reserve space for `bytes` from `src`; returns the offset in the block
    size_t push(const void* src, size_t bytes);
    // allocate the device block on `s`, copy, record the guard event.
    lc_status commit(hipStream_t s, void** dev_base);

  private:
    DeviceCtx* ctx_;
    std::vector<unsigned char> host_;
};

// Stream-ordered device allocation (hipMallocAsync / hipFreeAsync on the
// device's default pool, whose release threshold is raised at set-up).
lc_status dev_alloc(void** p, size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

// A stream-ordered device buffer that is freed on its stream when it goes
// out of scope (or at reset()), so every early return releases what was
// allocated before it.
template <typename T>
class DevBuf {
  public:
    DevBuf() = default;
    ~DevBuf() { reset(); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    lc_status alloc(size_t n, hipStream_t s) {
        reset();
        s_ = s;
        return dev_alloc(reinterpret_cast<void**>(&p_), sizeof(T) * n, s);
    }
    void reset() {
        dev_free(p_, s_);
        p_ = nullptr;
    }
    T* get() const { return p_; }

  private:
    T* p_ = nullptr;
    hipStream_t s_ = nullptr;
};

// ---------------------------------------------------------------------------
// geometry shared by the mesh and the pair kernels
// ---------------------------------------------------------------------------
struct GridGeom {
    int32_t n[3];        // cells per axis
    int32_t lo[3];       // origin, coordinate units
    int64_t ext[3];      // extent per axis: periodic = box, open = hi - lo + 1
    int32_t periodic;
    int32_t box;
    int64_t ncell;       // n[0] * n[1] * n[2] coarse cells
    int32_t sub;         // sub-cells per axis inside a coarse cell (1, 2 or 4)
    int32_t nsub;        // sub^3
};

// Cell index along an axis: floor((x - lo) n / ext).
__host__ __device__ inline int32_t axis_cell(int32_t x, int32_t lo, int64_t ext, int32_t n) {
    return int32_t((int64_t(x - lo) * n) / ext);
}

// Integer origin of cell c along an axis: the smallest coordinate the cell
// can hold, lo + ceil(c ext / n).  Points are stored relative to it, so every
// stored coordinate lies in [0, ceil(ext / n)] and is exact in float32.
__host__ __device__ inline int64_t cell_origin(int32_t c, int32_t lo, int64_t ext, int32_t n) {
    return int64_t(lo) + (int64_t(c) * ext + n - 1) / n;
}

}  // namespace lc

// Opaque mesh handle (public name from lc.h).
struct lc_cells {
    int device = -1;
    int32_t n_cat = 0;
    int64_t n_total = 0;
    std::vector<int64_t> offsets;   // host copy [n_cat + 1]
    lc::GridGeom g{};
    int32_t los = 0;
    int64_t r_max = 0;              // largest r edge the mesh was built for
    float* pts = nullptr;           // sorted points, float32 (x, y, z) relative to their cell origin
    // starts of the sub-cells, [n_cat][ncell][nsub] + 1 (global point index);
    // coarse cell c of catalogue k spans [cs[(k ncell + c) nsub], cs[(k ncell + c + 1) nsub])
    int64_t* cs = nullptr;
    size_t bytes = 0;
};

namespace lc {
// Validates a binning (see lc.h); LC_OK or LC_ERR_INVALID / LC_ERR_RANGE.
lc_status check_binning(const lc_binning* b);

// Number of stencil offsets and the list itself for a mesh and r_max
// (pi_max > 0: the (r_p, pi) binning, r_max bounding r_p in x and y and
// pi_max bounding |s_z|).  Order: [0] = (0,0,0); then the lexicographically
// positive half; then the negative half.  Offsets whose cells cannot hold a
// counted pair are pruned.  Returns n_half (self + positive half).
int build_stencil(const GridGeom& g, int64_t r_max, int64_t pi_max, std::vector<int4>& out);
// Largest separation along any axis that a counted pair can have: r_max,
// or for the (r_p, pi) binning the larger of the r_p bound and pi_max.
int64_t mesh_reach(const lc_binning* b);

// Drop the cached pair-count graphs and autotuning results.
void release_graphs();
// Drop the cached graphs captured on one mesh (called when it is freed).
void forget_graphs(const lc_cells* cells);
void release_tuning();
}  // namespace lc
