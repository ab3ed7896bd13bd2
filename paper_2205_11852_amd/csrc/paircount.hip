// Pair counting in (r, mu) bins for many catalogue pairs at once: the DD,
// DR_i and RR_i counts of the split Landy-Szalay estimator (Sect. 2.1),
// binned as in Sect. 4.3.
//
// Work decomposition: a work item is (task, run of consecutive cells of
// catalogue a).  Items of all tasks form one queue that persistent wavefronts
// drain with an atomic counter.  For every cell a wave takes up to 64 points
// of catalogue a (one per lane, float64 in registers) and streams the points
// of each neighbour cell of catalogue b through wave-uniform (scalar) loads.
//
// Per candidate pair (phase A, all lanes): float64 separation and squared
// distance d2 -- exact, since coordinates are integers below 2^25 -- and the
// r-range test.  Accepted pairs are compacted into a per-wave LDS ring
// (ballot + mbcnt), so the binning (phase B) always runs on 64 live lanes.
// Phase B estimates the r and mu bins in float32 and keeps the estimate only
// when it is provably away from every bin edge (error bound derived in the
// host code that sets eps_r / eps_m); otherwise it decides with the exact
// integer rule (int64 squared edges, 128-bit mu cross-multiplication).
// The bin is added to a wave-private uint32 LDS histogram that is flushed
// with uint64 global atomics when the wave moves to another task.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>

#include "lc_internal.hpp"

namespace lc {

constexpr int kQ = 128;  // entries of the per-wave compaction ring

struct PcParams {
    int32_t nx, ny, nz, periodic;
    int64_t ncell;
    double boxd;
    int32_t nhalf, nfull;
    int32_t cells_per_item, items_per_task;
    int64_t n_items;
    int32_t single_task;
    int32_t n_r, n_mu, nbins;
    int32_t hist_stride;   // uint32 words per wave histogram
    int32_t wave_bytes;    // LDS bytes per wave
    double emin2, emax2;
    double e0d, ded;
    float e0f, inv_drf, nmuf, nmu_m1_eps, eps_r, eps_m;
    int32_t force_exact;
    int32_t pad_;
};

typedef unsigned __int128 u128;

__device__ __forceinline__ uint64_t sq64(int64_t v) { return uint64_t(v) * uint64_t(v); }

template <bool UNIFORM>
__device__ __forceinline__ int exact_r(double d2, int k_est, const PcParams& p,
                                       const double* __restrict__ e2tab) {
    if (UNIFORM) {
        const uint64_t D2 = uint64_t(d2);
        const int64_t e0 = int64_t(p.e0d), de = int64_t(p.ded);
        int k = min(max(k_est, 0), p.n_r - 1);
        while (k > 0 && D2 < sq64(e0 + int64_t(k) * de)) --k;
        while (k < p.n_r - 1 && D2 >= sq64(e0 + int64_t(k + 1) * de)) ++k;
        return k;
    } else {
        int lo = 0, hi = p.n_r;  // e2[lo] <= d2 < e2[hi]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (e2tab[mid] <= d2) lo = mid;
            else hi = mid;
        }
        return lo;
    }
}

// largest m in [0, n_mu-1] with m^2 * den <= num  (den > 0)
__device__ __forceinline__ int exact_mu(u128 den, u128 num, int m_est, int n_mu) {
    int m = min(max(m_est, 0), n_mu - 1);
    while (m > 0 && u128(uint64_t(m) * uint64_t(m)) * den > num) --m;
    while (m < n_mu - 1 && u128(uint64_t(m + 1) * uint64_t(m + 1)) * den <= num) ++m;
    return m;
}

// Bin of one pair.  LOS 0: a = dz.  LOS 1: a = p = s.l, b = q = l.l.
template <int LOS, bool UNIFORM>
__device__ __forceinline__ int bin_pair(double d2, double a, double b, const PcParams& p,
                                        const double* __restrict__ e2tab, bool& used_exact) {
    const float fd2 = float(d2);
    const float rs = __builtin_amdgcn_rsqf(fd2);
    float tm;
    if (LOS == 0) {
        tm = fabsf(float(a)) * rs * p.nmuf;
    } else {
        const float rq = __builtin_amdgcn_rsqf(float(b));
        tm = fabsf(float(a)) * rs * rq * p.nmuf;
    }
    // clamp before converting: NaN (d2 = 0 or q = 0) becomes 0 here and
    // fails the margin test below, which sends the pair to the integer rule
    int m = int(fminf(fmaxf(tm, 0.0f), p.nmuf));
    const float fm = tm - float(m);
    bool ok = (tm >= p.nmu_m1_eps) || ((fm > p.eps_m) && (fm < 1.0f - p.eps_m));
    int k;
    if (UNIFORM) {
        const float r = fd2 * rs;
        const float tr = (r - p.e0f) * p.inv_drf;
        k = int(fminf(fmaxf(tr, 0.0f), float(p.n_r)));
        const float fr = tr - float(k);
        ok = ok && (fr > p.eps_r) && (fr < 1.0f - p.eps_r) && (k < p.n_r);
    } else {
        k = exact_r<false>(d2, 0, p, e2tab);
    }
    ok = ok && !p.force_exact;
    m = min(m, p.n_mu - 1);
    used_exact = !ok;
    if (!ok) {
        if (UNIFORM) k = exact_r<true>(d2, k, p, e2tab);
        const uint64_t D2 = uint64_t(d2);
        const uint64_t nm2 = uint64_t(p.n_mu) * uint64_t(p.n_mu);
        if (LOS == 0) {
            const uint64_t AZ = uint64_t(fabs(a));
            m = (D2 == 0) ? 0 : exact_mu(u128(D2), u128(nm2) * AZ * AZ, m, p.n_mu);
        } else {
            const uint64_t AP = uint64_t(fabs(a)), Q = uint64_t(b);
            m = (D2 == 0 || Q == 0) ? 0 : exact_mu(u128(D2) * Q, u128(nm2) * AP * AP, m, p.n_mu);
        }
    }
    return k * p.n_mu + m;
}

struct WaveState {
    unsigned* hist;
    double2* qa;
    double* qb;
    uint32_t qhead, qtail;
    uint64_t since_flush;
    uint64_t n_cand, n_binned, n_exact, n_flush;
    int cur_task;
};

template <int LOS, bool UNIFORM>
__device__ __forceinline__ void drain(WaveState& w, int lane, uint32_t n, const PcParams& p,
                                      const double* __restrict__ e2tab) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (uint32_t(lane) < n) {
        const uint32_t pos = (w.qhead + lane) & (kQ - 1);
        const double2 e = w.qa[pos];
        const double b = (LOS == 1) ? w.qb[pos] : 0.0;
        bool ex;
        const int bin = bin_pair<LOS, UNIFORM>(e.x, e.y, b, p, e2tab, ex);
        __hip_atomic_fetch_add(&w.hist[bin], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        w.n_exact += __popcll(__ballot(ex));
    }
    w.qhead += n;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LOS, bool UNIFORM>
__device__ __forceinline__ void flush(WaveState& w, int lane, const PcParams& p,
                                      const double* __restrict__ e2tab,
                                      unsigned long long* __restrict__ counts) {
    const uint32_t left = w.qtail - w.qhead;
    if (left) drain<LOS, UNIFORM>(w, lane, left, p, e2tab);
    unsigned long long* dst = counts + int64_t(w.cur_task) * p.nbins;
    for (int b = lane; b < p.nbins; b += 64) {
        const unsigned v = w.hist[b];
        if (v) {
            __hip_atomic_fetch_add(dst + b, (unsigned long long)v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            w.hist[b] = 0;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    w.since_flush = 0;
    w.n_flush++;
}

// Stream the points j in [jb, je) of catalogue b against this lane's point.
template <int LOS, bool UNIFORM, bool HAS_EMIN, bool SELF>
__device__ __forceinline__ void scan_range(WaveState& w, int lane, int64_t jb, int64_t je, double sx,
                                           double sy, double sz, int64_t gi,
                                           const double4* __restrict__ pts, const PcParams& p,
                                           const double* __restrict__ e2tab,
                                           unsigned long long* __restrict__ counts) {
    for (int64_t j = jb; j < je; ++j) {
        const double4 q = pts[j];
        const double dx = q.x - sx, dy = q.y - sy, dz = q.z - sz;
        const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
        bool acc = d2 < p.emax2;
        if (HAS_EMIN) acc = acc && (d2 >= p.emin2);
        if (SELF) acc = acc && (j > gi);
        double va = dz, vb = 0.0;
        if (LOS == 1) {
            const double lx = q.x + sx, ly = q.y + sy, lz = q.z + sz;
            va = fma(dx, lx, fma(dy, ly, dz * lz));
            vb = fma(lx, lx, fma(ly, ly, lz * lz));
        }
        const unsigned long long bal = __ballot(acc);
        if (bal) {
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
            if (acc) {
                const uint32_t pos = (w.qtail + rank) & (kQ - 1);
                w.qa[pos] = make_double2(d2, va);
                if (LOS == 1) w.qb[pos] = vb;
            }
            const uint32_t nb = __popcll(bal);
            w.qtail += nb;
            w.n_binned += nb;
            w.since_flush += nb;
            if (w.qtail - w.qhead >= 64) drain<LOS, UNIFORM>(w, lane, 64, p, e2tab);
            // a uint32 bin can take at most this many more pairs before a flush
            if (w.since_flush >= 0xFFFF0000ull) flush<LOS, UNIFORM>(w, lane, p, e2tab, counts);
        }
    }
}

template <int LOS, bool UNIFORM, bool HAS_EMIN>
__global__ __launch_bounds__(512) void k_pair_count(
    const double4* __restrict__ pts, const int64_t* __restrict__ cs, const int2* __restrict__ tasks,
    const int32_t* __restrict__ order, const int4* __restrict__ sten, const double* __restrict__ e2tab,
    unsigned long long* __restrict__ counts, unsigned long long* __restrict__ stats,
    unsigned* __restrict__ queue, PcParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    unsigned char* wb = smem + size_t(wid) * p.wave_bytes;
    WaveState w;
    w.hist = reinterpret_cast<unsigned*>(wb);
    w.qa = reinterpret_cast<double2*>(wb + size_t(p.hist_stride) * 4);
    w.qb = reinterpret_cast<double*>(w.qa + kQ);
    w.qhead = w.qtail = 0;
    w.since_flush = 0;
    w.n_cand = w.n_binned = w.n_exact = w.n_flush = 0;
    w.cur_task = -1;
    for (int b = lane; b < p.hist_stride; b += 64) w.hist[b] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    for (;;) {
        unsigned item = 0;
        if (lane == 0) item = atomicAdd(queue, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (int64_t(item) >= p.n_items) break;
        int task, g;
        if (p.single_task >= 0) {
            task = p.single_task;
            g = int(item);
        } else {
            task = order[item / unsigned(p.items_per_task)];
            g = int(item % unsigned(p.items_per_task));
        }
        task = __builtin_amdgcn_readfirstlane(task);
        if (task != w.cur_task) {
            if (w.cur_task >= 0) flush<LOS, UNIFORM>(w, lane, p, e2tab, counts);
            w.cur_task = task;
        }
        const int2 tk = tasks[task];
        const bool autop = tk.x == tk.y;
        const int64_t abase = int64_t(tk.x) * p.ncell, bbase = int64_t(tk.y) * p.ncell;
        const int64_t c0 = int64_t(g) * p.cells_per_item;
        const int64_t c1 = min(c0 + p.cells_per_item, p.ncell);
        const int ns = autop ? p.nhalf : p.nfull;
        for (int64_t c = c0; c < c1; ++c) {
            const int64_t ia0 = cs[abase + c], ia1 = cs[abase + c + 1];
            if (ia0 == ia1) continue;
            const int cx = int(c % p.nx);
            const int64_t t = c / p.nx;
            const int cy = int(t % p.ny);
            const int cz = int(t / p.ny);
            for (int64_t ib = ia0; ib < ia1; ib += 64) {
                const int64_t gi = ib + lane;
                double xi = 1e30, yi = 1e30, zi = 1e30;
                if (gi < ia1) {
                    const double4 q = pts[gi];
                    xi = q.x;
                    yi = q.y;
                    zi = q.z;
                }
                const int64_t nvalid = min(int64_t(64), ia1 - ib);
                for (int s = 0; s < ns; ++s) {
                    const int4 o = sten[s];
                    int jx = cx + o.x, jy = cy + o.y, jz = cz + o.z;
                    double shx = 0.0, shy = 0.0, shz = 0.0;
                    if (p.periodic) {
                        if (jx < 0) { jx += p.nx; shx = -p.boxd; } else if (jx >= p.nx) { jx -= p.nx; shx = p.boxd; }
                        if (jy < 0) { jy += p.ny; shy = -p.boxd; } else if (jy >= p.ny) { jy -= p.ny; shy = p.boxd; }
                        if (jz < 0) { jz += p.nz; shz = -p.boxd; } else if (jz >= p.nz) { jz -= p.nz; shz = p.boxd; }
                    } else if (jx < 0 || jx >= p.nx || jy < 0 || jy >= p.ny || jz < 0 || jz >= p.nz) {
                        continue;
                    }
                    const int64_t jc = (int64_t(jz) * p.ny + jy) * p.nx + jx;
                    int64_t jb = cs[bbase + jc];
                    const int64_t je = cs[bbase + jc + 1];
                    const bool self = autop && s == 0;
                    if (self) jb = ib + 1;
                    if (jb >= je) continue;
                    w.n_cand += uint64_t(nvalid) * uint64_t(je - jb);
                    // image of point j: x_j + shift, so s = x_j - (x_i - shift)
                    const double sx = xi - shx, sy = yi - shy, sz = zi - shz;
                    if (self)
                        scan_range<LOS, UNIFORM, HAS_EMIN, true>(w, lane, jb, je, sx, sy, sz, gi, pts, p,
                                                                 e2tab, counts);
                    else
                        scan_range<LOS, UNIFORM, HAS_EMIN, false>(w, lane, jb, je, sx, sy, sz, gi, pts, p,
                                                                  e2tab, counts);
                }
            }
        }
    }
    if (w.cur_task >= 0) flush<LOS, UNIFORM>(w, lane, p, e2tab, counts);
    if (stats && lane == 0) {
        atomicAdd(&stats[0], (unsigned long long)w.n_cand);
        atomicAdd(&stats[1], (unsigned long long)w.n_binned);
        atomicAdd(&stats[2], (unsigned long long)w.n_exact);
        atomicAdd(&stats[3], (unsigned long long)w.n_flush);
    }
}

typedef void (*PcKernel)(const double4*, const int64_t*, const int2*, const int32_t*, const int4*,
                         const double*, unsigned long long*, unsigned long long*, unsigned*, PcParams);

static PcKernel pick_kernel(int los, bool uniform, bool has_emin) {
    static const PcKernel tab[2][2][2] = {
        {{k_pair_count<0, false, false>, k_pair_count<0, false, true>},
         {k_pair_count<0, true, false>, k_pair_count<0, true, true>}},
        {{k_pair_count<1, false, false>, k_pair_count<1, false, true>},
         {k_pair_count<1, true, false>, k_pair_count<1, true, true>}},
    };
    return tab[los][uniform ? 1 : 0][has_emin ? 1 : 0];
}

__global__ void k_zero_counters(unsigned* q, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) q[i] = 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct Plan {
    PcKernel kern;
    PcParams p;
    int threads;
    int blocks;          // persistent grid
    size_t lds;
    int mode;
    int n_tasks;
    std::vector<int> task_blocks;   // per-task grid (LC_PER_TASK)
    // staged device block layout
    std::vector<unsigned char> blob;
    size_t off_tasks, off_order, off_sten, off_e2, off_queue;
    int n_queue;
};

static float f32_up(double v) {  // float >= v
    float f = float(v);
    if (double(f) < v) f = std::nextafter(f, INFINITY);
    return f;
}

static lc_status make_plan(DeviceCtx* ctx, const lc_cells* cells, const lc_task* tasks, int32_t n_tasks,
                           const lc_binning* b, int32_t mode, const lc_tuning* tune, Plan& pl) {
    const GridGeom& g = cells->g;
    const int n_r = b->n_r, n_mu = b->n_mu;
    PcParams& p = pl.p;
    std::memset(&p, 0, sizeof p);
    p.nx = g.n[0];
    p.ny = g.n[1];
    p.nz = g.n[2];
    p.periodic = g.periodic;
    p.ncell = g.ncell;
    p.boxd = double(g.box);
    std::vector<int4> sten;
    const int64_t rmax = b->r_edges[n_r];
    p.nhalf = build_stencil(g, rmax, sten);
    p.nfull = int(sten.size());
    int cpi = tune && tune->cells_per_item > 0 ? tune->cells_per_item : 0;
    if (cpi <= 0) {
        // about 16 items per wave slot over the whole batch, at least one row of cells
        cpi = std::max(1, g.n[0]);
    }
    cpi = int(std::min<int64_t>(cpi, g.ncell));
    p.cells_per_item = cpi;
    p.items_per_task = int((g.ncell + cpi - 1) / cpi);
    p.n_r = n_r;
    p.n_mu = n_mu;
    p.nbins = n_r * n_mu;
    p.hist_stride = (p.nbins + 3) & ~3;
    const bool mid = b->los == LC_LOS_MID;
    p.wave_bytes = p.hist_stride * 4 + kQ * 16 + (mid ? kQ * 8 : 0);
    const int64_t e0 = b->r_edges[0];
    p.emin2 = double(e0) * double(e0);
    p.emax2 = double(rmax) * double(rmax);
    bool uniform = true;
    const int64_t de = b->r_edges[1] - b->r_edges[0];
    for (int k = 0; k <= n_r; k++)
        if (int64_t(b->r_edges[k]) != e0 + int64_t(k) * de) uniform = false;
    p.e0d = double(e0);
    p.ded = double(de);
    p.e0f = float(e0);
    p.inv_drf = float(1.0 / double(de));
    p.nmuf = float(n_mu);
    // Float32 error bounds (relative, in units of 2^-24):
    //  mu estimate  n_mu |s_z| rsq(d2): conversions 1 + 0.5, rsq 2, two products 2  -> 5.5
    //  (midpoint adds p, q conversions, a second rsq and a product: -> 10)
    //  r estimate   d2 * rsq(d2): 0.5 + 2 + 1 = 3.5 of r; then (r - e0) * (1/de): 3 more
    // The margins below are 4-6x these bounds; anything closer to an edge is
    // decided with integers.
    const double u = std::ldexp(1.0, -24);
    double em = (mid ? 10.0 : 5.5) * u * n_mu;
    p.eps_m = f32_up(std::max(4.0 * em, std::ldexp(1.0, -22)));
    p.nmu_m1_eps = f32_up(double(n_mu - 1) + double(p.eps_m));
    double er = 3.5 * u * double(rmax) / double(de) + 3.0 * u * double(n_r);
    p.eps_r = f32_up(std::max(4.0 * er, std::ldexp(1.0, -22)));
    p.force_exact = (mode & LC_FORCE_EXACT) ? 1 : 0;
    const bool has_emin = e0 > 0;
    pl.kern = pick_kernel(mid ? 1 : 0, uniform, has_emin);
    pl.mode = mode;
    pl.n_tasks = n_tasks;

    int wpb = tune && tune->waves_per_block > 0 ? tune->waves_per_block : 4;
    if (wpb != 1 && wpb != 2 && wpb != 4 && wpb != 8)
        return fail(LC_ERR_INVALID, "waves_per_block = %d, must be 1, 2, 4 or 8", wpb);
    while (wpb > 1 && size_t(wpb) * p.wave_bytes > ctx->max_lds_block) wpb >>= 1;
    pl.threads = wpb * 64;
    pl.lds = size_t(wpb) * p.wave_bytes;
    if (pl.lds > ctx->max_lds_block)
        return fail(LC_ERR_INVALID, "histogram of %d bins does not fit in LDS", p.nbins);
    if (pl.lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)pl.kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           int(pl.lds));
        if (e != hipSuccess) return fail(LC_ERR_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
    }
    int occ = 0;
    LC_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)pl.kern, pl.threads, pl.lds));
    occ = std::max(occ, 1);
    int bpc = tune && tune->blocks_per_cu > 0 ? std::min(tune->blocks_per_cu, occ) : occ;
    pl.blocks = ctx->n_cu * bpc;

    // task order: largest first (cost ~ n_a * n_b, halved for auto pairs)
    std::vector<int32_t> order(n_tasks);
    std::vector<double> cost(n_tasks);
    for (int t = 0; t < n_tasks; t++) {
        const int a = tasks[t].cat_a, bb = tasks[t].cat_b;
        const double na = double(cells->offsets[a + 1] - cells->offsets[a]);
        const double nb = double(cells->offsets[bb + 1] - cells->offsets[bb]);
        cost[t] = a == bb ? 0.5 * na * na : na * nb;
        order[t] = t;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    const int64_t n_items = int64_t(n_tasks) * p.items_per_task;
    if (n_items >= (int64_t(1) << 31))
        return fail(LC_ERR_OVERFLOW, "%lld work items exceed the 32-bit queue", (long long)n_items);
    const bool per_task = (mode & LC_PER_TASK) != 0;
    p.n_items = per_task ? p.items_per_task : n_items;
    p.single_task = -1;
    pl.n_queue = per_task ? n_tasks : 1;
    if (per_task) {
        pl.task_blocks.resize(n_tasks);
        for (int t = 0; t < n_tasks; t++) {
            int64_t need = (p.items_per_task + wpb - 1) / wpb;
            pl.task_blocks[t] = int(std::max<int64_t>(1, std::min<int64_t>(need, pl.blocks)));
        }
    }
    // staged block: tasks, order, stencil, squared edges, zeroed queue counters
    std::vector<double> e2(n_r + 1);
    for (int k = 0; k <= n_r; k++) e2[k] = double(b->r_edges[k]) * double(b->r_edges[k]);
    std::vector<unsigned> qz(pl.n_queue, 0u);
    auto put = [&](const void* src, size_t bytes) {
        size_t off = (pl.blob.size() + 255) & ~size_t(255);
        pl.blob.resize(off + bytes);
        if (bytes) std::memcpy(pl.blob.data() + off, src, bytes);
        return off;
    };
    pl.off_tasks = put(tasks, sizeof(lc_task) * n_tasks);
    pl.off_order = put(order.data(), sizeof(int32_t) * n_tasks);
    pl.off_sten = put(sten.data(), sizeof(int4) * sten.size());
    pl.off_e2 = put(e2.data(), sizeof(double) * e2.size());
    pl.off_queue = put(qz.data(), sizeof(unsigned) * qz.size());
    return LC_OK;
}

static void launch_plan(const Plan& pl, const lc_cells* cells, unsigned char* dev, uint64_t* counts,
                        uint64_t* stats, hipStream_t s) {
    const int2* d_tasks = reinterpret_cast<const int2*>(dev + pl.off_tasks);
    const int32_t* d_order = reinterpret_cast<const int32_t*>(dev + pl.off_order);
    const int4* d_sten = reinterpret_cast<const int4*>(dev + pl.off_sten);
    const double* d_e2 = reinterpret_cast<const double*>(dev + pl.off_e2);
    unsigned* d_q = reinterpret_cast<unsigned*>(dev + pl.off_queue);
    auto* c = reinterpret_cast<unsigned long long*>(counts);
    auto* st = reinterpret_cast<unsigned long long*>(stats);
    if (pl.mode & LC_PER_TASK) {
        PcParams p = pl.p;
        for (int t = 0; t < pl.n_tasks; t++) {
            p.single_task = t;
            hipLaunchKernelGGL(pl.kern, dim3(pl.task_blocks[t]), dim3(pl.threads), pl.lds, s, cells->pts,
                               cells->cs, d_tasks, d_order, d_sten, d_e2, c, st, d_q + t, p);
        }
    } else {
        hipLaunchKernelGGL(pl.kern, dim3(pl.blocks), dim3(pl.threads), pl.lds, s, cells->pts, cells->cs,
                           d_tasks, d_order, d_sten, d_e2, c, st, d_q, pl.p);
    }
}

// Graph cache: captured launch sequences keyed by everything they bake in.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    void* dev = nullptr;  // owned copy of the staged block
};
static std::mutex g_graph_mu;
static std::map<std::string, GraphEntry> g_graphs;

static std::string graph_key(const Plan& pl, const lc_cells* cells, uint64_t* counts, uint64_t* stats,
                             int device) {
    std::string k;
    auto add = [&](const void* p, size_t n) { k.append(reinterpret_cast<const char*>(p), n); };
    add(&device, sizeof device);
    add(&cells, sizeof cells);
    add(&counts, sizeof counts);
    add(&stats, sizeof stats);
    add(&pl.mode, sizeof pl.mode);
    add(&pl.p, sizeof pl.p);
    add(&pl.blocks, sizeof pl.blocks);
    add(&pl.threads, sizeof pl.threads);
    add(pl.blob.data(), pl.blob.size());
    return k;
}

static lc_status run_graph(const Plan& pl, const lc_cells* cells, uint64_t* counts, uint64_t* stats,
                           hipStream_t s, int device) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    const std::string key = graph_key(pl, cells, counts, stats, device);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        GraphEntry ge;
        LC_TRY_HIP(hipMalloc(&ge.dev, pl.blob.size()));
        LC_TRY_HIP(hipMemcpy(ge.dev, pl.blob.data(), pl.blob.size(), hipMemcpyHostToDevice));
        hipStream_t cap;
        LC_TRY_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            unsigned* d_q = reinterpret_cast<unsigned*>(static_cast<unsigned char*>(ge.dev) + pl.off_queue);
            // queue counters are cleared by a kernel node (no memset nodes)
            k_zero_counters<<<1, 256, 0, cap>>>(d_q, pl.n_queue);
            launch_plan(pl, cells, static_cast<unsigned char*>(ge.dev), counts, stats, cap);
            e = hipStreamEndCapture(cap, &ge.graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) {
            if (ge.graph) (void)hipGraphDestroy(ge.graph);
            (void)hipFree(ge.dev);
            return fail(LC_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
        }
        it = g_graphs.emplace(key, ge).first;
    }
    LC_TRY_HIP(hipGraphLaunch(it->second.exec, s));
    return LC_OK;
}

void release_graphs() {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& kv : g_graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        if (kv.second.dev) (void)hipFree(kv.second.dev);
    }
    g_graphs.clear();
}

}  // namespace lc

using namespace lc;

extern "C" lc_status lc_pair_count_batch(const lc_cells* cells, const lc_task* tasks, int32_t n_tasks,
                                         const lc_binning* b, uint64_t* counts, int32_t mode,
                                         const lc_tuning* tune, uint64_t* stats, void* stream) {
    clear_error();
    if (!cells) return fail(LC_ERR_INVALID, "cells is NULL");
    LC_TRY(check_binning(b));
    if (n_tasks < 0) return fail(LC_ERR_INVALID, "n_tasks < 0");
    if (n_tasks == 0) return LC_OK;
    if (!tasks) return fail(LC_ERR_INVALID, "tasks is NULL");
    if (!counts) return fail(LC_ERR_INVALID, "counts is NULL");
    const int base_mode = mode & ~(LC_GRAPH | LC_FORCE_EXACT);
    if (base_mode != LC_PERSISTENT && base_mode != LC_PER_TASK)
        return fail(LC_ERR_INVALID, "mode = %d is not LC_PERSISTENT or LC_PER_TASK (| flags)", mode);
    if (b->periodic != cells->g.periodic || (b->periodic && b->box_units != cells->g.box))
        return fail(LC_ERR_INVALID, "binning geometry differs from the mesh's");
    for (int32_t t = 0; t < n_tasks; t++)
        if (tasks[t].cat_a < 0 || tasks[t].cat_a >= cells->n_cat || tasks[t].cat_b < 0 ||
            tasks[t].cat_b >= cells->n_cat)
            return fail(LC_ERR_INVALID, "task %d has catalogue ids (%d, %d) outside [0, %d)", t,
                        tasks[t].cat_a, tasks[t].cat_b, cells->n_cat);
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    if (ctx->device != cells->device) return fail(LC_ERR_INVALID, "mesh lives on another device");
    Plan pl;
    LC_TRY(make_plan(ctx, cells, tasks, n_tasks, b, mode, tune, pl));
    hipStream_t s = (hipStream_t)stream;
    if (mode & LC_GRAPH) return run_graph(pl, cells, counts, stats, s, ctx->device);
    void* dev = nullptr;
    {
        Stager stg(ctx);
        stg.push(pl.blob.data(), pl.blob.size());
        LC_TRY(stg.commit(s, &dev));
    }
    launch_plan(pl, cells, static_cast<unsigned char*>(dev), counts, stats, s);
    hipError_t e = hipGetLastError();
    dev_free(dev, s);
    if (e != hipSuccess) return fail(LC_ERR_HIP, "pair-count launch failed: %s", hipGetErrorString(e));
    return LC_OK;
}
