// Chaining mesh: counting sort of every catalogue into one shared grid of
// cells, so that pair counting only visits cells that can hold pairs closer
// than r_max.  Steps: (open geometry) bounding box -> cell id and per-cell
// histogram -> exclusive scan -> scatter of the points as float32 values
// relative to their cell's integer origin -> a fixed order inside each
// sub-cell.
#include <algorithm>
#include <cmath>

#include "lc_internal.hpp"

namespace lc {

static constexpr int kLimit24 = 1 << 24;

lc_status check_binning(const lc_binning* b) {
    if (!b) return fail(LC_ERR_INVALID, "binning is NULL");
    if (!b->r_edges) return fail(LC_ERR_INVALID, "binning.r_edges is NULL");
    if (b->n_r < 1) return fail(LC_ERR_INVALID, "n_r = %d, must be >= 1", b->n_r);
    if (b->n_mu < 1 || b->n_mu > LC_MAX_NMU)
        return fail(LC_ERR_INVALID, "n_mu = %d, must be in [1, %d]", b->n_mu, LC_MAX_NMU);
    if ((int64_t)b->n_r * b->n_mu > LC_MAX_BINS)
        return fail(LC_ERR_INVALID, "n_r * n_mu = %lld exceeds %d", (long long)b->n_r * b->n_mu,
                    LC_MAX_BINS);
    if (b->periodic != 0 && b->periodic != 1)
        return fail(LC_ERR_INVALID, "periodic = %d, must be 0 or 1", b->periodic);
    if (b->los != LC_LOS_Z && b->los != LC_LOS_MID && b->los != LC_LOS_RPPI)
        return fail(LC_ERR_INVALID, "los = %d, must be LC_LOS_Z, LC_LOS_MID or LC_LOS_RPPI", b->los);
    if (b->los == LC_LOS_MID && b->periodic)
        return fail(LC_ERR_INVALID, "the midpoint line of sight needs open geometry");
    if (b->los == LC_LOS_RPPI && (b->pi_max < 1 || b->pi_max >= kLimit24))
        return fail(LC_ERR_INVALID, "pi_max = %d, must be in [1, 2^24) for LC_LOS_RPPI", b->pi_max);
    if (b->r_edges[0] < 0) return fail(LC_ERR_INVALID, "r_edges[0] = %d < 0", b->r_edges[0]);
    for (int k = 0; k < b->n_r; k++)
        if (b->r_edges[k + 1] <= b->r_edges[k])
            return fail(LC_ERR_INVALID, "r_edges not strictly increasing at %d", k);
    const int64_t rmax = mesh_reach(b);
    if (b->periodic) {
        if (b->box_units < 2 || b->box_units > kLimit24 || (b->box_units & 1))
            return fail(LC_ERR_INVALID, "box_units = %d must be even and in [2, 2^24]", b->box_units);
        if (2 * rmax >= b->box_units)
            return fail(LC_ERR_RANGE, "r_max = %lld must be < box/2 = %d", (long long)rmax,
                        b->box_units / 2);
    } else if (rmax >= (int64_t(1) << 25)) {
        return fail(LC_ERR_RANGE, "r_max = %lld must be < 2^25 in open geometry", (long long)rmax);
    }
    return LC_OK;
}

int64_t mesh_reach(const lc_binning* b) {
    const int64_t r = b->r_edges[b->n_r];
    return b->los == LC_LOS_RPPI ? std::max<int64_t>(r, b->pi_max) : r;
}

int build_stencil(const GridGeom& g, int64_t r_max, int64_t pi_max, std::vector<int4>& out) {
    // Two cells whose indices differ by d along an axis are more than
    // (|d| - 1) * w apart on it (w = ext / n).  Isotropic: an offset with
    // sum max(|d|-1, 0)^2 w^2 >= r_max^2 cannot hold a pair with r < r_max.
    // (r_p, pi): the sum runs over x and y only (against r_max, the r_p
    // bound), and max(|d_z|-1, 0) w_z >= pi_max rules out |s_z| < pi_max.
    // Decided exactly: multiply through by the n_a^2 in 128-bit integers.
    typedef unsigned __int128 u128;
    const bool rppi = pi_max > 0;
    const int nax = rppi ? 2 : 3;  // axes in the squared-distance sum
    int k[3];
    u128 wt[3];  // ext_a^2 * prod_{b != a, b < nax} n_b^2
    u128 rhs = u128(uint64_t(r_max)) * uint64_t(r_max);
    for (int a = 0; a < nax; a++) rhs *= u128(uint64_t(g.n[a])) * uint64_t(g.n[a]);
    for (int a = 0; a < 3; a++) {
        wt[a] = u128(uint64_t(g.ext[a])) * uint64_t(g.ext[a]);
        for (int b = 0; b < nax; b++)
            if (b != a) wt[a] *= u128(uint64_t(g.n[b])) * uint64_t(g.n[b]);
        // smallest |d| with (|d| - 1) * w >= reach, capped: one full turn of a
        // periodic grid (or the whole open grid) reaches every cell
        const int64_t reach = (rppi && a == 2) ? pi_max : r_max;
        int64_t kk = (reach * g.n[a]) / g.ext[a] + 1;
        k[a] = int(std::min<int64_t>(kk, g.n[a]));
    }
    std::vector<int4> pos, neg;
    for (int dz = -k[2]; dz <= k[2]; dz++)
        for (int dy = -k[1]; dy <= k[1]; dy++)
            for (int dx = -k[0]; dx <= k[0]; dx++) {
                if (!dx && !dy && !dz) continue;
                const int d[3] = {dx, dy, dz};
                u128 s = 0;
                for (int a = 0; a < nax; a++) {
                    const uint64_t m = uint64_t(std::max(std::abs(d[a]) - 1, 0));
                    s += u128(m * m) * wt[a];
                }
                if (s >= rhs) continue;
                if (rppi) {
                    // (|d_z| - 1) ext_z / n_z >= pi_max, exactly
                    const int64_t mz = std::max(std::abs(dz) - 1, 0);
                    if (mz * g.ext[2] >= pi_max * int64_t(g.n[2])) continue;
                }
                const bool positive = dz > 0 || (dz == 0 && (dy > 0 || (dy == 0 && dx > 0)));
                (positive ? pos : neg).push_back(make_int4(dx, dy, dz, 0));
            }
    out.clear();
    out.push_back(make_int4(0, 0, 0, 0));
    out.insert(out.end(), pos.begin(), pos.end());
    const int n_half = int(out.size());
    out.insert(out.end(), neg.begin(), neg.end());
    return n_half;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// floor(num / den) for 0 <= num < 2^53 and 0 < den, given rden = 1 / den in
// float64: the float64 estimate lies within one of the quotient, and one
// exact step corrects it (a 64-bit integer division is a long instruction
// sequence on the GPU).
__device__ inline int64_t floordiv_est(int64_t num, int64_t den, double rden) {
    int64_t q = int64_t(double(num) * rden);
    if (q * den > num) --q;
    else if ((q + 1) * den <= num) ++q;
    return q;
}

// axis_cell and cell_origin on the device, with rext = 1 / ext and rn = 1 / n
__device__ inline int32_t axis_cell_d(int32_t x, int32_t lo, int64_t ext, int32_t n, double rext) {
    return int32_t(floordiv_est(int64_t(x - lo) * n, ext, rext));
}
__device__ inline int64_t cell_origin_d(int32_t c, int32_t lo, int64_t ext, int32_t n, double rn) {
    return int64_t(lo) + floordiv_est(int64_t(c) * ext + n - 1, n, rn);
}

// Bounding box of all points (open geometry) and the |x| < 2^24 check.
__global__ void k_bbox(const int32_t* __restrict__ xyz, int64_t n, int32_t* __restrict__ box,
                       unsigned* __restrict__ err) {
    int mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    bool bad = false;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; a++) {
            int v = xyz[a * n + p];
            mn[a] = min(mn[a], v);
            mx[a] = max(mx[a], v);
            bad |= (v <= -kLimit24) || (v >= kLimit24);
        }
    }
    for (int a = 0; a < 3; a++) {
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = min(mn[a], __shfl_xor(mn[a], o));
            mx[a] = max(mx[a], __shfl_xor(mx[a], o));
        }
    }
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 3; a++) {
            atomicMin(&box[a], mn[a]);
            atomicMax(&box[3 + a], mx[a]);
        }
    }
    if (bad) atomicOr(err, 1u);
}

__global__ void k_fill_box(int32_t* box) {
    if (threadIdx.x < 3) box[threadIdx.x] = INT32_MAX;
    else if (threadIdx.x < 6) box[threadIdx.x] = INT32_MIN;
}

__global__ void k_zero_u32(unsigned* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Catalogue lookup: lut[b] is the last catalogue starting at or before
// point b << kCatShift (built on the host); a point's catalogue is found
// from there by skipping forward past catalogues that end at or before it.
constexpr int kCatShift = 12;

__device__ __forceinline__ int32_t find_cat(const int64_t* __restrict__ off, const int32_t* __restrict__ lut,
                                            int64_t p) {
    int32_t c = lut[p >> kCatShift];
    while (off[c + 1] <= p) ++c;  // ends: p < off[n_cat]
    return c;
}

// Cell id per point, its arrival rank within the sub-cell (the returned
// value of the per-cell counter, which varies from run to run), packed as
// id << 32 | rank (sub-cell ids are below 2^31), and the per-cell histogram;
// range check for periodic boxes (an out-of-range point gets ~0).
__global__ void k_cell_count(const int32_t* __restrict__ xyz, int64_t n, const int64_t* __restrict__ off,
                             const int32_t* __restrict__ lut, GridGeom g, uint64_t* __restrict__ gid,
                             unsigned* __restrict__ cnt, unsigned* __restrict__ err) {
    const double r0 = 1.0 / double(g.ext[0]), r1 = 1.0 / double(g.ext[1]), r2 = 1.0 / double(g.ext[2]);
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        int32_t x = xyz[p], y = xyz[n + p], z = xyz[2 * n + p];
        if (g.periodic) {
            if (x < 0 || y < 0 || z < 0 || x >= g.box || y >= g.box || z >= g.box) {
                atomicOr(err, 2u);
                gid[p] = ~0ull;
                continue;
            }
        }
        // fine index along each axis; coarse cell = fine / sub (the floors nest)
        const int32_t fx = axis_cell_d(x, g.lo[0], g.ext[0], g.n[0] * g.sub, r0);
        const int32_t fy = axis_cell_d(y, g.lo[1], g.ext[1], g.n[1] * g.sub, r1);
        const int32_t fz = axis_cell_d(z, g.lo[2], g.ext[2], g.n[2] * g.sub, r2);
        const int32_t cx = fx / g.sub, cy = fy / g.sub, cz = fz / g.sub;
        const int32_t sid = ((fz - cz * g.sub) * g.sub + (fy - cy * g.sub)) * g.sub + (fx - cx * g.sub);
        const int32_t c = find_cat(off, lut, p);
        const int64_t id = (int64_t(c) * g.ncell + (int64_t(cz) * g.n[1] + cy) * g.n[0] + cx) * g.nsub + sid;
        const unsigned rank = atomicAdd(&cnt[id], 1u);
        gid[p] = (uint64_t(id) << 32) | rank;
    }
}

// Exclusive scan of uint32 cell counts into int64 starts.
static constexpr int kScanThreads = 256;
static constexpr int kScanItems = 8;
static constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; w++) {
        if (w < wid) base += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__global__ void k_scan_reduce(const unsigned* __restrict__ cnt, int64_t n, int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int64_t s = 0;
    for (int i = 0; i < kScanItems; i++)
        if (base + i < n) s += cnt[base + i];
    int64_t tot;
    (void)block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_top(int64_t* __restrict__ bsum, int64_t nb, int64_t* __restrict__ grand) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        int64_t i = b0 + threadIdx.x;
        int64_t v = i < nb ? bsum[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ void k_scan_down(const unsigned* __restrict__ cnt, int64_t n, const int64_t* __restrict__ boff,
                            int64_t* __restrict__ out) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    unsigned v[kScanItems];
    int64_t s = 0;
    for (int i = 0; i < kScanItems; i++) {
        v[i] = base + i < n ? cnt[base + i] : 0u;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, sh, &tot) + boff[blockIdx.x];
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n) out[base + i] = ex;
        ex += v[i];
    }
}

__global__ void k_scan_last(int64_t* out, int64_t n, const int64_t* grand) { out[n] = *grand; }

struct F3 {
    float x, y, z;
};

// Scatter: each point, as float32 offsets from its coarse cell's integer
// origin, goes to its sub-cell's slot for its arrival rank: one 12-byte
// store into the mesh, or (STAGE, for a fixed order) a 16-byte record with
// the sub-cell id as its fourth word into the staging array.
template <bool STAGE>
__global__ void k_scatter(const int32_t* __restrict__ xyz, int64_t n, const uint64_t* __restrict__ gid,
                          const int64_t* __restrict__ cs, GridGeom g, void* __restrict__ out) {
    double rext[3], rn[3];
    for (int a = 0; a < 3; a++) {
        rext[a] = 1.0 / double(g.ext[a]);
        rn[a] = 1.0 / double(g.n[a]);
    }
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t gv = gid[p];
        if (gv == ~0ull) continue;
        const int64_t slot = cs[int64_t(gv >> 32)] + int64_t(uint32_t(gv));
        const int32_t v[3] = {xyz[p], xyz[n + p], xyz[2 * n + p]};
        float r[3];
        for (int a = 0; a < 3; a++) {
            const int32_t c = axis_cell_d(v[a], g.lo[a], g.ext[a], g.n[a], rext[a]);
            r[a] = float(int64_t(v[a]) - cell_origin_d(c, g.lo[a], g.ext[a], g.n[a], rn[a]));
        }
        if (STAGE)
            static_cast<float4*>(out)[slot] = make_float4(r[0], r[1], r[2], __int_as_float(int32_t(gv >> 32)));
        else
            static_cast<F3*>(out)[slot] = F3{r[0], r[1], r[2]};
    }
}

// Fixed order inside every sub-cell (the default; lc_mesh_opts.arrival_order
// skips it): the point in staging slot t goes to rank = the number of its
// sub-cell's points that precede it in (x, y, z) order, points with equal
// coordinates ranked by slot; equal points are the same three floats, so the
// stored mesh does not depend on the arrival order.  Each point reads its
// whole sub-cell (consecutive slots, so the lanes of a wave mostly read the
// same record): quadratic in the sub-cell's size, like the pair count's own
// work there.
__device__ __forceinline__ int before(const float4 q, const float4 me, int rq, int rm) {
    return q.x < me.x || (q.x == me.x && (q.y < me.y || (q.y == me.y && (q.z < me.z ||
                                                                        (q.z == me.z && rq < rm)))));
}

__global__ void k_order(int64_t ntot_cells, const int64_t* __restrict__ cs, const float4* __restrict__ stage,
                        F3* __restrict__ pts) {
    // slots [0, cs[ntot_cells]) are filled (a periodic point out of the box
    // has none: that build fails after this launch)
    const int64_t n = cs[ntot_cells];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const float4 me = stage[t];
        const int64_t id = __float_as_int(me.w);
        const int64_t s0 = cs[id];
        const float4* seg = stage + s0;
        const int c = int(cs[id + 1] - s0), my = int(t - s0);
        int rank = 0, u = 0;
        for (; u + 4 <= c; u += 4) {
            const float4 q0 = seg[u], q1 = seg[u + 1], q2 = seg[u + 2], q3 = seg[u + 3];
            rank += before(q0, me, u, my) + before(q1, me, u + 1, my) + before(q2, me, u + 2, my) +
                    before(q3, me, u + 3, my);
        }
        for (; u < c; u++) rank += before(seg[u], me, u, my);
        pts[s0 + rank] = F3{me.x, me.y, me.z};
    }
}

static int grid_for(int64_t n, int threads, int n_cu) {
    int64_t b = (n + threads - 1) / threads;
    int64_t cap = int64_t(n_cu) * 16;
    return int(std::max<int64_t>(1, std::min(b, cap)));
}

}  // namespace lc

using namespace lc;

static void free_cells_mem(lc_cells* c) {
    if (!c) return;
    if (c->pts) (void)hipFree(c->pts);
    if (c->cs) (void)hipFree(c->cs);
    c->pts = nullptr;
    c->cs = nullptr;
}

extern "C" void lc_free_cells(lc_cells* cells) {
    if (!cells) return;
    forget_graphs(cells);
    free_cells_mem(cells);
    delete cells;
}

extern "C" lc_status lc_cells_get_info(const lc_cells* c, lc_cells_info* info) {
    clear_error();
    if (!c || !info) return fail(LC_ERR_INVALID, "NULL argument");
    info->n_cat = c->n_cat;
    info->sub = c->g.sub;
    info->reserved = 0;
    for (int a = 0; a < 3; a++) {
        info->grid[a] = c->g.n[a];
        info->cell_side[a] = double(c->g.ext[a]) / double(c->g.n[a]);
    }
    info->n_total = c->n_total;
    info->bytes = (int64_t)c->bytes;
    return LC_OK;
}

extern "C" lc_status lc_build_cells(const int32_t* xyz, int64_t n_total, const int64_t* cat_offsets,
                                    int32_t n_cat, const lc_binning* b, const lc_mesh_opts* opts,
                                    void* stream, lc_cells** out) {
    clear_error();
    if (!out) return fail(LC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    LC_TRY(check_binning(b));
    const int32_t cell_units = opts ? opts->cell_units : 0;
    int32_t sub = opts && opts->sub ? opts->sub : 2;
    const int32_t arrival_order = opts ? opts->arrival_order : 0;
    if (sub != 1 && sub != 2 && sub != 4) return fail(LC_ERR_INVALID, "sub = %d, must be 1, 2 or 4", sub);
    if (arrival_order != 0 && arrival_order != 1)
        return fail(LC_ERR_INVALID, "arrival_order = %d, must be 0 or 1", arrival_order);
    const bool fixed_order = arrival_order == 0;
    if (n_cat < 1) return fail(LC_ERR_INVALID, "n_cat = %d, must be >= 1", n_cat);
    if (!cat_offsets) return fail(LC_ERR_INVALID, "cat_offsets is NULL");
    if (n_total < 0) return fail(LC_ERR_INVALID, "n_total < 0");
    if (n_total > 0 && !xyz) return fail(LC_ERR_INVALID, "xyz is NULL");
    if (cell_units < 0) return fail(LC_ERR_INVALID, "cell_units < 0");
    if (cat_offsets[0] != 0) return fail(LC_ERR_INVALID, "cat_offsets[0] != 0");
    for (int32_t c = 0; c < n_cat; c++)
        if (cat_offsets[c + 1] < cat_offsets[c])
            return fail(LC_ERR_INVALID, "cat_offsets decreasing at %d", c);
    if (cat_offsets[n_cat] != n_total) return fail(LC_ERR_INVALID, "cat_offsets[n_cat] != n_total");
    if (n_total >= (int64_t(1) << 40)) return fail(LC_ERR_OVERFLOW, "n_total too large");
    for (int32_t c = 0; c < n_cat; c++)
        if (cat_offsets[c + 1] - cat_offsets[c] >= kMaxCatalogue)
            return fail(LC_ERR_OVERFLOW, "catalogue %d holds %lld points; a catalogue holds fewer than %lld",
                        c, (long long)(cat_offsets[c + 1] - cat_offsets[c]), (long long)kMaxCatalogue);

    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    hipStream_t s = (hipStream_t)stream;
    const int64_t rmax = mesh_reach(b);

    GridGeom g{};
    g.periodic = b->periodic;
    g.box = b->periodic ? b->box_units : 0;
    DevBuf<unsigned> errb;  // [0] error word, [8..13] bounding box
    LC_TRY(errb.alloc(16, s));
    unsigned* d_err = errb.get();
    k_zero_u32<<<1, 64, 0, s>>>(d_err, 16);
    if (b->periodic) {
        for (int a = 0; a < 3; a++) {
            g.lo[a] = 0;
            g.ext[a] = b->box_units;
        }
    } else {
        int32_t* d_box = (int32_t*)(d_err + 8);
        k_fill_box<<<1, 64, 0, s>>>(d_box);
        if (n_total > 0)
            k_bbox<<<grid_for(n_total, 256, ctx->n_cu), 256, 0, s>>>(xyz, n_total, d_box, d_err);
        unsigned h[16];
        LC_TRY_HIP(hipMemcpyAsync(h, d_err, sizeof h, hipMemcpyDeviceToHost, s));
        LC_TRY_HIP(hipStreamSynchronize(s));
        if (h[0] & 1u) return fail(LC_ERR_RANGE, "a coordinate is outside |x| < 2^24");
        const int32_t* hb = (const int32_t*)(h + 8);
        for (int a = 0; a < 3; a++) {
            if (n_total == 0) {
                g.lo[a] = 0;
                g.ext[a] = 1;
            } else {
                g.lo[a] = hb[a];
                g.ext[a] = int64_t(hb[3 + a]) - hb[a] + 1;
            }
        }
    }

    // cell side: requested, or about 96 points per cell of a mean catalogue,
    // kept within [r_max / 3, r_max]
    double vol = double(g.ext[0]) * double(g.ext[1]) * double(g.ext[2]);
    double w;
    if (cell_units > 0) {
        w = cell_units;
    } else {
        double nbar = std::max(1.0, double(n_total) / n_cat);
        w = std::cbrt(vol * 96.0 / nbar);
        w = std::min(std::max(w, double(rmax) / 3.0), double(rmax));
    }
    w = std::max(w, 1.0);
    for (;;) {
        g.ncell = 1;
        for (int a = 0; a < 3; a++) {
            int64_t na = int64_t(std::floor(double(g.ext[a]) / w));
            na = std::max<int64_t>(1, std::min<int64_t>(na, 1024));
            g.n[a] = int32_t(na);
            g.ncell *= na;
        }
        if (g.ncell * int64_t(n_cat) <= (int64_t(1) << 28)) break;
        w *= 1.25;
    }
    // sub-cells: at least 1 unit wide, and at most 2^31 starts in all
    for (int a = 0; a < 3; a++)
        while (sub > 1 && g.ext[a] / (int64_t(g.n[a]) * sub) < 1) sub /= 2;
    while (sub > 1 && g.ncell * int64_t(n_cat) * sub * sub * sub > (int64_t(1) << 31)) sub /= 2;
    g.sub = sub;
    g.nsub = sub * sub * sub;

    auto* cells = new lc_cells();
    cells->device = ctx->device;
    cells->n_cat = n_cat;
    cells->n_total = n_total;
    cells->offsets.assign(cat_offsets, cat_offsets + n_cat + 1);
    cells->g = g;
    cells->los = b->los;
    cells->r_max = rmax;
    const int64_t ntot_cells = g.ncell * int64_t(n_cat) * g.nsub;
    // 4 extra points of padding: pair counting reads whole groups of four
    size_t pts_bytes = size_t(std::max<int64_t>(n_total, 1) + 4) * 3 * sizeof(float);
    size_t cs_bytes = size_t(ntot_cells + 1) * sizeof(int64_t);
    if (hipMalloc(&cells->pts, pts_bytes) != hipSuccess || hipMalloc(&cells->cs, cs_bytes) != hipSuccess) {
        (void)hipGetLastError();
        free_cells_mem(cells);
        delete cells;
        return fail(LC_ERR_NOMEM, "mesh allocation (%zu + %zu bytes) failed", pts_bytes, cs_bytes);
    }
    cells->bytes = pts_bytes + cs_bytes;

    // temporaries
    int64_t* d_off = nullptr;
    const int32_t* d_lut = nullptr;
    uint64_t* d_gid = nullptr;
    float4* d_stage = nullptr;
    unsigned* d_cnt = nullptr;
    int64_t* d_bsum = nullptr;
    const int64_t nblk = (ntot_cells + kScanTile - 1) / kScanTile;
    lc_status st = LC_OK;
    {
        // catalogue of every (1 << kCatShift)-th point: the last catalogue
        // starting at or before it
        std::vector<int32_t> lut(size_t(n_total >> kCatShift) + 1);
        int32_t c = 0;
        for (size_t bi = 0; bi < lut.size(); bi++) {
            const int64_t p0 = int64_t(bi) << kCatShift;
            while (c + 1 < n_cat && cat_offsets[c + 1] <= p0) ++c;
            lut[bi] = c;
        }
        Stager stg(ctx);
        stg.push(cat_offsets, sizeof(int64_t) * (n_cat + 1));
        const size_t lut_off = stg.push(lut.data(), sizeof(int32_t) * lut.size());
        st = stg.commit(s, (void**)&d_off);
        if (st == LC_OK) d_lut = reinterpret_cast<const int32_t*>(reinterpret_cast<unsigned char*>(d_off) + lut_off);
    }
    if (st == LC_OK) st = dev_alloc((void**)&d_gid, sizeof(uint64_t) * std::max<int64_t>(n_total, 1), s);
    if (st == LC_OK && fixed_order)
        st = dev_alloc((void**)&d_stage, sizeof(float4) * std::max<int64_t>(n_total, 1), s);
    if (st == LC_OK) st = dev_alloc((void**)&d_cnt, sizeof(unsigned) * ntot_cells, s);
    if (st == LC_OK) st = dev_alloc((void**)&d_bsum, sizeof(int64_t) * (nblk + 1), s);
    if (st != LC_OK) {
        dev_free(d_off, s);
        dev_free(d_gid, s);
        dev_free(d_stage, s);
        dev_free(d_cnt, s);
        dev_free(d_bsum, s);
        lc_free_cells(cells);
        return st;
    }
    k_zero_u32<<<grid_for(ntot_cells, 256, ctx->n_cu), 256, 0, s>>>(d_cnt, ntot_cells);
    // the padding after the last point reads as zeros
    k_zero_u32<<<1, 64, 0, s>>>(reinterpret_cast<unsigned*>(cells->pts) + 3 * n_total, 12);
    if (n_total > 0)
        k_cell_count<<<grid_for(n_total, 256, ctx->n_cu), 256, 0, s>>>(xyz, n_total, d_off, d_lut, g,
                                                                       d_gid, d_cnt, d_err);
    k_scan_reduce<<<nblk, kScanThreads, 0, s>>>(d_cnt, ntot_cells, d_bsum);
    k_scan_top<<<1, kScanThreads, 0, s>>>(d_bsum, nblk, d_bsum + nblk);
    k_scan_down<<<nblk, kScanThreads, 0, s>>>(d_cnt, ntot_cells, d_bsum, cells->cs);
    k_scan_last<<<1, 1, 0, s>>>(cells->cs, ntot_cells, d_bsum + nblk);
    if (n_total > 0 && fixed_order) {
        k_scatter<true><<<grid_for(n_total, 256, ctx->n_cu), 256, 0, s>>>(xyz, n_total, d_gid, cells->cs, g,
                                                                          d_stage);
        k_order<<<grid_for(n_total, 256, ctx->n_cu), 256, 0, s>>>(ntot_cells, cells->cs, d_stage,
                                                                  reinterpret_cast<F3*>(cells->pts));
    } else if (n_total > 0) {
        k_scatter<false><<<grid_for(n_total, 256, ctx->n_cu), 256, 0, s>>>(xyz, n_total, d_gid, cells->cs,
                                                                           g, cells->pts);
    }
    unsigned herr = 0;
    hipError_t e = hipMemcpyAsync(&herr, d_err, sizeof herr, hipMemcpyDeviceToHost, s);
    dev_free(d_off, s);
    dev_free(d_gid, s);
    dev_free(d_stage, s);
    dev_free(d_cnt, s);
    dev_free(d_bsum, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        lc_free_cells(cells);
        return fail(LC_ERR_HIP, "mesh build failed: %s", hipGetErrorString(e));
    }
    if (herr & 2u) {
        lc_free_cells(cells);
        return fail(LC_ERR_RANGE, "a coordinate is outside the periodic box [0, %d)", g.box);
    }
    *out = cells;
    return LC_OK;
}
