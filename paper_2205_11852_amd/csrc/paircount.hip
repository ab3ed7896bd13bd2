// Pair counting in (r, mu) bins for many catalogue pairs at once: the DD,
// DR_i and RR_i counts of the split Landy-Szalay estimator (Sect. 2.1),
// binned as in Sect. 4.3 (or in (r_p, pi) for the projected correlation
// function, Sect. 2.3).
//
// Data: every catalogue is sorted into a shared chaining mesh; points are
// stored as float32 (x, y, z) relative to their cell's integer origin, so
// every stored value and every difference formed below is an integer below
// 2^24 in magnitude and exact in float32.
//
// Work decomposition: a work item is (task, run of consecutive cells of
// catalogue a).  Items form eight queues, one per XCD (workgroup w runs on
// XCD w mod 8), each holding a contiguous, cost-balanced range of tasks so
// that the blocks sharing an XCD's L2 share catalogues; a block whose queue
// is empty moves on to the next queue.  A block takes one item at a time and
// its waves share the item's stencil offsets.  For each chunk of i points
// (up to a whole cell of catalogue a, read through wave-uniform scalar
// loads), a wave gathers the points of the kept neighbour sub-cells of
// catalogue b into blocks of 64, one per lane.
//
// Phase A (every candidate, all lanes): separation and a float32 squared
// distance, accepted against r_max with a margin larger than its rounding
// error; accepted pairs are compacted into a per-wave LDS queue
// (ballot + mbcnt), so phase B always runs on 64 live lanes.
// Phase B: float32 estimates of the r and mu bins, kept only when they lie
// farther from every bin edge than their proven error (eps_r, eps_m, derived
// in make_plan); every other pair goes to a second per-wave queue and is
// decided by the integer rule (exact squared distances and edges, mu by
// exact cross-multiplication), which also drops pairs that phase A's margin
// let through.  The midpoint line of sight reads each pair's x_j from a
// per-wave LDS table of the swept j points' absolute coordinates.  Bins go
// to an LDS histogram shared by the block's waves (uint32 bins, or two
// 16-bit bins per word for large binnings, each wrap corrected in the
// counts at once), flushed with uint64 global atomics when the block moves
// to another task.
#include <climits>
#include <cstddef>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>

#include "lc_internal.hpp"

namespace lc {

constexpr int kQ = 128;     // entries of the per-wave compaction queue
static_assert(kQ >= 127, "a drain reads queue slots up to 63 + 63");
constexpr int kX = 128;     // entries of the per-wave queue of pairs for the integer rule
constexpr int kX16 = 64;    // the same with 16-bit bins (less LDS per wave, more waves per CU)
constexpr int kXm = 32;     // the same for the midpoint line of sight (32-byte entries)
constexpr int kJ = 128;     // midpoint: rows of the per-wave j table (the swept block, then carried pairs)
// entries of the integer-rule queue and its bytes per wave
constexpr int kx_for(int los, bool h16) { return los == 1 ? kXm : h16 ? kX16 : kX; }
constexpr int kx_bytes(int los, bool h16) { return kx_for(los, h16) * (los == 1 ? 32 : 16); }
constexpr int kXcd = 8;     // queues (one per XCD)

struct PcParams {
    int32_t n[3];
    int32_t periodic;
    int32_t lo[3];
    int32_t single_task;
    int64_t ext[3];
    int64_t box;
    int64_t ncell;
    int32_t sub, nsub;          // sub-cells per axis / per coarse cell
    float wf[3];                // sub-cell side per axis (ext / (n sub))
    int32_t pad1;
    int32_t nhalf, nfull;
    int32_t cells_per_item, items_per_task;
    int32_t chunk, pad3;        // i points per chunk (multiple of 4, <= 64)
    int32_t n_r, n_mu, nbins;
    int32_t hist_stride;    // uint32 words of the block histogram (bins + a discard slot)
    int32_t queue_byte0;    // LDS byte offset of wave 0's queue
    int32_t pad2;
    float emax2_hi, emin2_lo;   // phase A acceptance (float32, with margin)
    float inv_drf, nmuf;
    // estimates shifted down by their margins and the single-compare bounds
    // on their fractions (see bin_fast)
    float r_shift, ok_r, mu_shift, ok_m;
    float pimax_f;              // (r_p, pi) binning: |s_z| bound (an exact integer)
    uint32_t nmu4;              // bytes per r row of the histogram: 4 n_mu (2 n_mu with 16-bit bins)
    uint32_t h16_init;          // 16-bit bins: initial value of a histogram word (two bins)
    uint32_t wave_limit;        // candidate tests a wave may register between flushes
    uint32_t qstart[kXcd + 1];  // queue x holds items [qstart[x], qstart[x+1])
};

typedef unsigned __int128 u128;

// Constants of the integer rule.  Kept in device memory and read only on that
// (rare) path, so that they hold no registers in the loops.
struct ExactTab {
    int64_t emin2, emax2;   // exact squared outer edges
    int64_t e0, de;         // uniform edges: e_k = e0 + k de
    int32_t n_r, n_mu;
    int32_t discard;        // histogram slot of dropped pairs (= n_r n_mu)
    int32_t pad;
    int64_t pi_max;         // (r_p, pi) binning: |s_z| bound
    int64_t e2[1];          // [n_r + 1] squared edges (flexible tail)
};

// A value every lane holds equally, made visible as such to the compiler so
// that loads indexed by it become scalar loads.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ uint64_t sq64(int64_t v) { return uint64_t(v * v); }

// largest m in [0, n_mu-1] with m^2 * den <= num  (den > 0)
__device__ __forceinline__ int exact_mu(u128 den, u128 num, int m_est, int n_mu) {
    int m = min(max(m_est, 0), n_mu - 1);
    while (m > 0 && u128(uint64_t(m) * uint64_t(m)) * den > num) --m;
    while (m < n_mu - 1 && u128(uint64_t(m + 1) * uint64_t(m + 1)) * den <= num) ++m;
    return m;
}

// a * b <= c * d, exactly, for float64 operands whose products do not
// underflow: each product is p + (fma(a, b, -p)) exactly, and rounding is
// monotonic, so the pairs (p, low part) order like the exact products.
__device__ __forceinline__ bool prod_le(double a, double b, double c, double d) {
    const double p = a * b, q = c * d;
    if (p != q) return p < q;
    return fma(a, b, -p) <= fma(c, d, -q);
}

// Integer rule for the plane-parallel line of sight, in float64: the
// separation components are integers below 2^25, so their squares and d^2
// (below 2^52), the squared edges and m^2, n_mu^2 (below 2^20) are exact;
// the mu test m^2 d^2 <= n_mu^2 s_z^2 is decided exactly by prod_le.
template <bool UNIFORM>
__device__ __forceinline__ int exact_bin_z(double x, double y, double z, int k_est, int m_est,
                                           const ExactTab* __restrict__ xt) {
    const double D2 = fma(x, x, fma(y, y, z * z));
    if (D2 >= double(xt->emax2) || D2 < double(xt->emin2)) return xt->discard;
    const int n_r = xt->n_r, n_mu = xt->n_mu;
    int k;
    if (UNIFORM) {
        const double e0 = double(xt->e0), de = double(xt->de);
        k = min(max(k_est, 0), n_r - 1);
        while (k > 0 && D2 < (e0 + k * de) * (e0 + k * de)) --k;
        while (k < n_r - 1 && D2 >= (e0 + (k + 1) * de) * (e0 + (k + 1) * de)) ++k;
    } else {
        int lo = 0, hi = n_r;  // e2[lo] <= D2 < e2[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (double(xt->e2[mid]) <= D2) lo = mid;
            else hi = mid;
        }
        k = lo;
    }
    int m = 0;
    if (D2 > 0.0) {
        const double nm2 = double(n_mu) * double(n_mu), z2 = z * z;
        m = min(max(m_est, 0), n_mu - 1);
        while (m > 0 && !prod_le(double(m) * double(m), D2, nm2, z2)) --m;
        while (m < n_mu - 1 && prod_le(double(m + 1) * double(m + 1), D2, nm2, z2)) ++m;
    }
    return k * n_mu + m;
}

// Integer rule for the (r_p, pi) binning, in float64 (exact: the components
// are integers below 2^25): r_p^2 = s_x^2 + s_y^2 against the squared edges,
// pi bin = floor(n_pi |s_z| / pi_max) for |s_z| < pi_max.
template <bool UNIFORM>
__device__ __forceinline__ int exact_bin_rppi(double x, double y, double z, int k_est,
                                              const ExactTab* __restrict__ xt) {
    const double RP2 = fma(x, x, y * y);
    const int64_t az = int64_t(fabs(z));
    if (RP2 >= double(xt->emax2) || RP2 < double(xt->emin2) || az >= xt->pi_max) return xt->discard;
    const int n_r = xt->n_r, n_mu = xt->n_mu;
    int k;
    if (UNIFORM) {
        const double e0 = double(xt->e0), de = double(xt->de);
        k = min(max(k_est, 0), n_r - 1);
        while (k > 0 && RP2 < (e0 + k * de) * (e0 + k * de)) --k;
        while (k < n_r - 1 && RP2 >= (e0 + (k + 1) * de) * (e0 + (k + 1) * de)) ++k;
    } else {
        int lo = 0, hi = n_r;  // e2[lo] <= RP2 < e2[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (double(xt->e2[mid]) <= RP2) lo = mid;
            else hi = mid;
        }
        k = lo;
    }
    return k * n_mu + int((int64_t(n_mu) * az) / xt->pi_max);
}

// Integer rule (the binning of Sect. 4.3 with exact comparisons): the bin of
// separation s (midpoint: P = s.l, Q = l.l), or the discard slot outside
// [e_0, e_n).
template <int LOS, bool UNIFORM>
__device__ __forceinline__ int exact_bin(int64_t sx, int64_t sy, int64_t sz, int64_t P, uint64_t Q,
                                         int k_est, int m_est, const ExactTab* __restrict__ xt) {
    const uint64_t D2 = sq64(sx) + sq64(sy) + sq64(sz);
    if (D2 >= uint64_t(xt->emax2) || D2 < uint64_t(xt->emin2)) return xt->discard;
    const int n_r = xt->n_r, n_mu = xt->n_mu;
    int k;
    if (UNIFORM) {
        const int64_t e0 = xt->e0, de = xt->de;
        k = min(max(k_est, 0), n_r - 1);
        while (k > 0 && D2 < sq64(e0 + int64_t(k) * de)) --k;
        while (k < n_r - 1 && D2 >= sq64(e0 + int64_t(k + 1) * de)) ++k;
    } else {
        int lo = 0, hi = n_r;  // e2[lo] <= D2 < e2[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (uint64_t(xt->e2[mid]) <= D2) lo = mid;
            else hi = mid;
        }
        k = lo;
    }
    const uint64_t nm2 = uint64_t(n_mu) * uint64_t(n_mu);
    int m;
    if (LOS == 0) {
        const uint64_t AZ = uint64_t(sz < 0 ? -sz : sz);
        m = (D2 == 0) ? 0 : exact_mu(u128(D2), u128(nm2) * AZ * AZ, m_est, n_mu);
    } else {
        const uint64_t AP = uint64_t(P < 0 ? -P : P);
        m = (D2 == 0 || Q == 0) ? 0 : exact_mu(u128(D2) * Q, u128(nm2) * AP * AP, m_est, n_mu);
    }
    return k * n_mu + m;
}

// A wave-uniform value held in a vector register.  The kernel keeps more
// live scalars than the scalar register file holds, and a spilled scalar is
// reloaded with v_readlane, one vector instruction per use; the constants of
// the innermost loops cost nothing extra as vector operands.
__device__ __forceinline__ float vreg(float x) {
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}
__device__ __forceinline__ uint32_t vreg(uint32_t x) {
    uint32_t r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// Constants of the binning of queued pairs held in vector registers (the
// midpoint kernel; the others read them from the parameters).
struct BinConst {
    float mu_shift, ok_m;
    uint32_t nmu4;
};

struct WaveState {
    BinConst bc;
    unsigned long long* dst;  // 16-bit bins: the current task's counts (wrap corrections)
    int32_t nbins;            // 16-bit bins: bins of a task (slots past it are the discard slot)
    unsigned* hist;       // the block's histogram (shared by its waves)
    float4* qa;           // this wave's queue of (sx, sy, sz, d2 | i index), entries [0, qtail)
    uint32_t qbyte;       // LDS slot of qa[0] (its byte offset / 16, in a vector register)
    const float* pj;      // points of the task's j catalogue (wave-uniform)
    uint32_t jbyte;       // midpoint: LDS byte offset of the j table: absolute x, y, z of a j point
                          // per 12-byte row; rows [0, 64) the swept block (row = lane), row 64 + q
                          // the j point of queue slot q carried over from earlier blocks
    int64_t b0;           // global index of the j catalogue's first point
    float4* xa;           // this wave's queue of pairs for the integer rule, entries [0, xn)
    float4* xj;           // midpoint: the absolute x, y, z of each of those pairs' j point
    uint32_t xn;          // wave-uniform
    uint32_t qtail;       // wave-uniform
    uint32_t since_flush; // candidate tests this wave registered since its last flush
    uint64_t n_cand;
    uint32_t n_exact;     // per lane: pairs binned by the integer rule
    uint32_t n_flush;     // block flushes (task changes), counted by thread 0
    uint32_t n_wflush;    // this wave's overflow-guard flushes
};

extern __shared__ __align__(16) unsigned char smem[];

// The LDS word at byte offset `off` of the dynamic block, addressed as the
// plain 32-bit LDS address `off`: the pair-count kernel has no static LDS
// (make_plan checks this), so its dynamic block starts at LDS address 0.
// A histogram slot k 4 n_mu + 4 m then costs one 24-bit multiply-add.
typedef __attribute__((address_space(3))) unsigned lds_u32_t;
__device__ __forceinline__ lds_u32_t* lds_u32_at(uint32_t off) { return (lds_u32_t*)(__UINTPTR_TYPE__)off; }
typedef __attribute__((address_space(3))) float lds_f32_t;
__device__ __forceinline__ lds_f32_t* lds_f32_at(uint32_t off) { return (lds_f32_t*)(__UINTPTR_TYPE__)off; }
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f32x4 lds_f4_t;
__device__ __forceinline__ lds_f4_t* lds_f4_at(uint32_t off) { return (lds_f4_t*)(__UINTPTR_TYPE__)off; }

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS byte address (in the block histogram at offset 0) of one queued pair's
// bin from its float32 estimates, and the fractions fm (mu) and fr (r) that
// decide whether the estimates are kept: only when fm < ok_m and fr < ok_r,
// i.e. farther than eps from every edge; otherwise the pair takes the
// integer rule later.  d2 = 0 (and q = 0) give NaN or clamped estimates that
// fail the test, so every value stays finite.  (A bound below 0 sends every
// pair to the integer rule.)
template <int LOS, bool UNIFORM, bool HAS_E0, bool FULL, bool H16>
__device__ __forceinline__ uint32_t bin_fast(const float4 e, uint32_t jbyte, const PcParams& p, const BinConst& bc,
                                             float& fm, float& fr, float3& xj) {
    // Each estimate is shifted down by its margin eps inside the FMA that
    // forms it, x' = x - eps.  Then fract(x') < 1 - 2 eps (one compare)
    // holds only when x lies in (floor(x') + eps', floor(x') + 1 - eps') with
    // eps' = eps minus the estimate's own error, i.e. strictly inside the
    // bin floor(x').  A shifted value below 0 (x within eps of 0) has a
    // fraction near 1 and fails, and so does NaN.  The scale constants are
    // folded into rsq(d2) first, so each FMA reads one scalar operand.
    float d2f, u, rs;
    if (LOS == 0) {
        d2f = e.w;
        rs = __builtin_amdgcn_rsqf(d2f);
        u = fmaf(fabsf(e.z), rs * p.nmuf, -p.mu_shift);
    } else if (LOS == 2) {
        // (r_p, pi): e.w = r_p^2; |s_z| is an exact integer and nmuf holds
        // n_pi / pi_max, so the pi estimate is one fma
        d2f = e.w;
        rs = __builtin_amdgcn_rsqf(d2f);
        u = fmaf(fabsf(e.z), p.nmuf, -p.mu_shift);
    } else {
        // l = x_i + x_j = 2 x_j - s from the j point's absolute coordinates
        // (returned in xj for the integer rule), read from the wave's j table
        // at the row e.w names.  A full drain reads 64 live entries; a
        // partial one masks the row so that a lane past the drained entries
        // (masked by the caller) reads inside the table.  l, p = s.l and
        // q = l.l in float32, within the error bound that make_plan's mu
        // margin covers.  d2 = 0 or q = 0 give an infinite rsq and a NaN
        // estimate, which fails.
        const uint32_t jl = FULL ? uint32_t(__float_as_int(e.w)) : (uint32_t(__float_as_int(e.w)) & uint32_t(kJ - 1));
        const lds_f32_t* row = lds_f32_at(jbyte + jl * 12u);
        xj = make_float3(row[0], row[1], row[2]);
        const float lx = fmaf(2.0f, xj.x, -e.x);
        const float ly = fmaf(2.0f, xj.y, -e.y);
        const float lz = fmaf(2.0f, xj.z, -e.z);
        const float P = fmaf(e.x, lx, fmaf(e.y, ly, e.z * lz));
        const float Q = fmaf(lx, lx, fmaf(ly, ly, lz * lz));
        d2f = fmaf(e.x, e.x, fmaf(e.y, e.y, e.z * e.z));
        rs = __builtin_amdgcn_rsqf(d2f);
        u = fmaf(fabsf(P) * (rs * p.nmuf), __builtin_amdgcn_rsqf(Q), -bc.mu_shift);
    }
    // |mu| n_mu <= n_mu exactly; an estimate within eps_m of n_mu (mu near 1)
    // fails the test, so m < n_mu whenever the pair is kept
    const uint32_t m = uint32_t(int(u));
    fm = __builtin_amdgcn_fractf(u);
    uint32_t k = 0;
    fr = 2.0f;  // non-uniform edges: fails every bound, the integer rule bins
    if (UNIFORM) {
        // eps_r also covers phase A's acceptance margin, so a pair outside
        // [e_0, e_n) never passes the test with k outside [0, n_r)
        const float t = fmaf(d2f, rs * p.inv_drf, -p.r_shift);
        k = uint32_t(int(t));
        fr = __builtin_amdgcn_fractf(t);
    }
    // 24-bit multiply-add: k < n_r and 4 n_mu are far below 2^24
    return __umul24(k, LOS == 1 ? bc.nmu4 : p.nmu4) + (m << (H16 ? 1 : 2));
}

// Histogram slot of one queued pair by the integer rule (discard slot when it
// lies outside [e_0, e_n)); the float64 estimates only seed the searches.
template <int LOS, bool UNIFORM>
__device__ __forceinline__ int exact_entry(const float4 e, const float4 xj, const ExactTab* __restrict__ xt) {
    const double x = e.x, y = e.y, z = e.z;
    const double d2 = fma(x, x, fma(y, y, z * z));
    const double r = sqrt(d2);
    if (LOS == 2) {
        const double rp = sqrt(fma(x, x, y * y));
        const int kp_est = UNIFORM ? int((rp - double(xt->e0)) / double(xt->de)) : 0;
        return exact_bin_rppi<UNIFORM>(x, y, z, kp_est, xt);
    }
    const int k_est = UNIFORM ? int((r - double(xt->e0)) / double(xt->de)) : 0;
    if (LOS == 0) {
        const int m_est = d2 > 0.0 ? int(fabs(z) / r * double(xt->n_mu)) : 0;
        return exact_bin_z<UNIFORM>(x, y, z, k_est, m_est, xt);
    }
    // exact: absolute coordinates (xj, of the j point) and separations are
    // integers, l below 2^26
    const double lx = 2.0 * double(xj.x) - x;
    const double ly = 2.0 * double(xj.y) - y;
    const double lz = 2.0 * double(xj.z) - z;
    const double P = fma(x, lx, fma(y, ly, z * lz));
    const double Q = fma(lx, lx, fma(ly, ly, lz * lz));
    const int m_est = (d2 > 0.0 && Q > 0.0) ? int(fabs(P) / sqrt(d2 * Q) * double(xt->n_mu)) : 0;
    return exact_bin<LOS, UNIFORM>(int64_t(int(e.x)), int64_t(int(e.y)), int64_t(int(e.z)), int64_t(P),
                                   uint64_t(Q), k_est, m_est, xt);
}

// A 16-bit bin wrapped from 65535 to 0: add its lost 65536 to the task's
// counts.  Bins 2t (low half) and 2t + 1 (high half) share LDS word t, so a
// wrap of the low half also carried one into the high half, whose count then
// loses it again; and if that carry wrapped the high half, the high bin lost
// 65536 too.  Every wrap is seen by exactly the atomic add that caused it (it
// returns the word's old value), so the corrections are exact whatever the
// order of the adds; the uint64 counts take -1 as 2^64 - 1.
__device__ __noinline__ void h16_wrap(const WaveState& w, uint32_t slot, uint32_t sh, uint32_t old) {
    const uint32_t lo = slot & ~1u, hi = lo + 1;
    unsigned long long* d = w.dst;
    const uint32_t nb = uint32_t(w.nbins);
    if (sh == 0) {
        if (lo < nb) __hip_atomic_fetch_add(d + lo, 65536ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (hi < nb) {
            const unsigned long long c = (old >> 16) == 0xFFFFu ? 65535ull : ~0ull;
            __hip_atomic_fetch_add(d + hi, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (hi < nb) {
        __hip_atomic_fetch_add(d + hi, 65536ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Add one to the histogram slot at LDS byte address `addr` (the histogram
// starts at address 0): a 32-bit bin, or with H16 a 16-bit half of a word.
template <bool H16>
__device__ __forceinline__ void hist_add(const WaveState& w, uint32_t addr) {
    if (!H16) {
        __hip_atomic_fetch_add(lds_u32_at(addr), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        const uint32_t sh = (addr & 2u) << 3;
        const uint32_t old =
            __hip_atomic_fetch_add(lds_u32_at(addr & ~3u), 1u << sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (((old >> sh) & 0xFFFFu) == 0xFFFFu) h16_wrap(w, addr >> 1, sh, old);
    }
}

// Bin the last n (<= 64) of the xn pairs waiting for the integer rule, one
// per lane with every lane busy.  Returns the new length.
template <int LOS, bool UNIFORM, bool H16>
__device__ __forceinline__ uint32_t drain_exact(WaveState& w, int lane, uint32_t n, uint32_t xn,
                                                const ExactTab* __restrict__ xt) {
    wave_sync_lds();
    const uint32_t first = xn - n;
    if (uint32_t(lane) < n) {
        const int bin = exact_entry<LOS, UNIFORM>(w.xa[first + lane], LOS == 1 ? w.xj[first + lane] : float4{}, xt);
        hist_add<H16>(w, uint32_t(bin) << (H16 ? 1 : 2));
        w.n_exact++;
    }
    wave_sync_lds();
    return __builtin_amdgcn_readfirstlane(first);
}

// Bin the last n (<= 64) of the qt queued pairs, one per lane (the queue is
// an unordered bag, so taking from its end leaves the rest in place).  Pairs
// the estimates cannot decide move to the integer-rule queue, which is binned
// 64 at a time.  Returns the new queue length.  Every lane reads a slot:
// first + lane stays inside the queue (a full drain starts at most 63
// entries in, since the queue held fewer than 64 before the last append of
// at most 64; a partial drain starts at 0), and lanes past n are masked.
// FULL: n = 64, so every slot read holds an entry of the current task.
template <int LOS, bool UNIFORM, bool HAS_E0, bool FULL, bool H16>
__device__ __forceinline__ uint32_t drain(WaveState& w, int lane, uint32_t n, uint32_t qt, const PcParams& p,
                                          const ExactTab* __restrict__ xt) {
    wave_sync_lds();
    const uint32_t first = qt - n;
    const float4 e = w.qa[first + lane];
    float fm, fr;
    float3 xj = make_float3(0.0f, 0.0f, 0.0f);
    const uint32_t addr = bin_fast<LOS, UNIFORM, HAS_E0, FULL, H16>(e, w.jbyte, p, w.bc, fm, fr, xj);
    const float ok_m = LOS == 1 ? w.bc.ok_m : p.ok_m;
    const bool live = uint32_t(lane) < n;
    const unsigned long long live_mask = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    // The lanes the estimates do not decide, from the two compares' lane
    // masks combined on the scalar unit (predicate 4 = ordered less-than, so
    // NaN fails).  The compiler shares these compares with the ones that
    // mask the histogram add; a ballot of the combined bool would copy the
    // mask through a vector register first.
    const unsigned long long xb =
        live_mask & ~(__builtin_amdgcn_fcmpf(fm, ok_m, 4) & __builtin_amdgcn_fcmpf(fr, p.ok_r, 4));
    const bool ok = (fm < ok_m) && (fr < p.ok_r);
    if (ok && live) hist_add<H16>(w, addr);
    if (xb) {
        uint32_t xn = __builtin_amdgcn_readfirstlane(w.xn);
        const uint32_t nx = uint32_t(__popcll(xb));
        // a queue shorter than 128 (16-bit bins, midpoint): a queue that
        // would pass it is binned first
        constexpr uint32_t cap = uint32_t(kx_for(LOS, H16));
        constexpr uint32_t batch = cap < 64u ? cap : 64u;
        if (cap < 128u && xn + nx > cap) xn = drain_exact<LOS, UNIFORM, H16>(w, lane, xn, xn, xt);
        if (cap < 64u && nx > cap) {
            // (midpoint) more of them than the queue holds: bin them here
            if (live && !ok) {
                const int bin = exact_entry<LOS, UNIFORM>(e, make_float4(xj.x, xj.y, xj.z, 0.0f), xt);
                hist_add<H16>(w, uint32_t(bin) << (H16 ? 1 : 2));
                w.n_exact++;
            }
        } else {
            if (live && !ok) {
                const uint32_t rank =
                    __builtin_amdgcn_mbcnt_hi(uint32_t(xb >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(xb), 0u));
                w.xa[xn + rank] = e;
                // (midpoint: with its j point's coordinates, since the j
                // table changes before the queue is binned)
                if (LOS == 1) w.xj[xn + rank] = make_float4(xj.x, xj.y, xj.z, 0.0f);
            }
            xn = __builtin_amdgcn_readfirstlane(xn + nx);
            if (xn >= batch) xn = drain_exact<LOS, UNIFORM, H16>(w, lane, batch, xn, xt);
        }
        w.xn = xn;
    }
    wave_sync_lds();
    return __builtin_amdgcn_readfirstlane(first);
}

// Bin everything this wave has queued (both queues).
template <int LOS, bool UNIFORM, bool HAS_E0, bool H16>
__device__ __forceinline__ void drain_all(WaveState& w, int lane, const PcParams& p,
                                          const ExactTab* __restrict__ xt) {
    if (w.qtail) w.qtail = drain<LOS, UNIFORM, HAS_E0, false, H16>(w, lane, w.qtail, w.qtail, p, xt);
    if (w.xn) w.xn = drain_exact<LOS, UNIFORM, H16>(w, lane, w.xn, w.xn, xt);
}

// Add the two 16-bit bins of histogram word t (slots 2t, 2t + 1) to the
// task's counts, less the value each bin started from (h16_init's halves;
// nonzero only in the wrap test mode), modulo 2^64.
__device__ __forceinline__ void h16_flush_word(uint32_t v, uint32_t init, int t, int nbins,
                                               unsigned long long* __restrict__ dst) {
    const unsigned long long lo = (v & 0xFFFFu), lo0 = (init & 0xFFFFu);
    const unsigned long long hi = (v >> 16), hi0 = (init >> 16);
    if (lo != lo0) __hip_atomic_fetch_add(dst + 2 * t, lo - lo0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (hi != hi0 && 2 * t + 1 < nbins)
        __hip_atomic_fetch_add(dst + 2 * t + 1, hi - hi0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every bin value is at most the sum over the block's waves of the candidate
// tests each registered since its last flush; each wave keeps its own share
// below 2^32 / waves, so no uint32 bin can wrap.  A wave whose share would
// pass that bound bins its queue and then moves the whole histogram out with
// atomic exchanges: counts other waves add meanwhile stay in the bins, and
// their shares still cover them.
template <int LOS, bool UNIFORM, bool HAS_E0, bool H16>
__device__ __forceinline__ void wave_flush(WaveState& w, int lane, const PcParams& p,
                                           const ExactTab* __restrict__ xt,
                                           unsigned long long* __restrict__ dst) {
    drain_all<LOS, UNIFORM, HAS_E0, H16>(w, lane, p, xt);
    if (!H16) {
        for (int b = lane; b < p.nbins; b += 64) {
            const unsigned v = __hip_atomic_exchange(&w.hist[b], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (v) __hip_atomic_fetch_add(dst + b, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else {
        // both halves of every word move out together; a half that wraps
        // meanwhile is corrected by its own add (h16_wrap)
        for (int t = lane; 2 * t < p.nbins; t += 64) {
            const unsigned v =
                __hip_atomic_exchange(&w.hist[t], p.h16_init, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            h16_flush_word(v, p.h16_init, t, p.nbins, dst);
        }
    }
    w.since_flush = 0;
    w.n_wflush++;
}

// End of a task: every wave has binned its queue; the block adds the
// histogram into the task's counts and clears it.  Called by all threads.
template <bool H16>
__device__ __forceinline__ void block_flush(unsigned* hist, int nbins, uint32_t h16_init,
                                            unsigned long long* __restrict__ dst) {
    __syncthreads();
    if (!H16) {
        for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
            const unsigned v = hist[b];
            if (v) {
                __hip_atomic_fetch_add(dst + b, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                hist[b] = 0;
            }
        }
    } else {
        for (int t = threadIdx.x; 2 * t < nbins; t += blockDim.x) {
            const unsigned v = hist[t];
            if (v != h16_init) {
                h16_flush_word(v, h16_init, t, nbins, dst);
                hist[t] = h16_init;
            }
        }
    }
    __syncthreads();
}

struct Cand {
    float dx, dy, dz, d2;
    bool acc;
};

// Separation and float32 squared distance of one candidate; accepted when
// d2 < e_max^2 (1 + 2^-20), which holds for every pair with r < e_max since
// the float32 sum of three exact squares is within 3 * 2^-24 of d2.  The
// (r_p, pi) binning (LOS 2) tests r_p^2 = s_x^2 + s_y^2 the same way and
// |s_z| < pi_max exactly (both are integers below 2^24).
template <int LOS, bool HAS_EMIN>
__device__ __forceinline__ Cand test_pair(float xj, float yj, float zj, float xi, float yi, float zi,
                                          const PcParams& p) {
    Cand c;
    c.dx = xj - xi;
    c.dy = yj - yi;
    c.dz = zj - zi;
    if (LOS == 2) {
        c.d2 = fmaf(c.dx, c.dx, c.dy * c.dy);
        c.acc = (c.d2 < p.emax2_hi) && (fabsf(c.dz) < p.pimax_f);
    } else {
        c.d2 = fmaf(c.dx, c.dx, fmaf(c.dy, c.dy, c.dz * c.dz));
        c.acc = c.d2 < p.emax2_hi;
    }
    if (HAS_EMIN) c.acc = c.acc && (c.d2 >= p.emin2_lo);
    return c;
}

// Append the accepted lanes of one candidate to the queue (length qt, kept
// wave-uniform); bin 64 of them as soon as 64 are queued.  w4: the j point's
// row of the j table (midpoint); the other modes queue d2 (r_p^2).
template <int LOS, bool UNIFORM, bool HAS_E0, bool H16>
__device__ __forceinline__ uint32_t push(WaveState& w, int lane, const Cand& c, float w4, unsigned long long bal,
                                         uint32_t qt, const PcParams& p, const ExactTab* __restrict__ xt) {
    qt = __builtin_amdgcn_readfirstlane(qt);
    if (bal) {
        if (c.acc) {
            // slot qt + (accepted lanes below this one).  The queue's first
            // slot sits in a vector register, where the lane count (mbcnt)
            // adds it as its accumulator, and one shift-add forms the LDS
            // address: the scalar unit, nearly as busy as the vector one
            // here, only scales qt (the compiler's own form added the base
            // on the scalar unit and shifted and added twice more)
            const float4 v = make_float4(c.dx, c.dy, c.dz, LOS == 1 ? w4 : c.d2);
            const uint32_t slot =
                __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), w.qbyte));
            uint32_t addr;
            asm("v_lshl_add_u32 %0, %1, 4, %2" : "=v"(addr) : "v"(slot), "s"(qt * 16u));
            *lds_f4_at(addr) = f32x4{v.x, v.y, v.z, v.w};
        }
        qt = __builtin_amdgcn_readfirstlane(qt + uint32_t(__popcll(bal)));
        if (qt >= 64) qt = drain<LOS, UNIFORM, HAS_E0, true, H16>(w, lane, 64, qt, p, xt);
    }
    return qt;
}

// Midpoint line of sight: this lane's j point of the block about to be swept
// (i cell frame x, y, z) goes into row `lane` of the wave's j table as
// absolute coordinates, the i cell's integer origin (ox, oy, oz) added back:
// integers below 2^24, so the sums are exact.  The binning reads them from
// LDS; queued pairs name the row.  Lanes without a point write values no
// queued pair names.
template <int LOS>
__device__ __forceinline__ void stage_j(const WaveState& w, int lane, float x, float y, float z, float ox,
                                        float oy, float oz) {
    if (LOS != 1) return;
    lds_f32_t* row = lds_f32_at(w.jbyte + uint32_t(lane) * 12u);
    row[0] = x + ox;
    row[1] = y + oy;
    row[2] = z + oz;
}

// Midpoint: after a block's sweep, the pairs still queued (fewer than 64, in
// slots [0, qtail)) that name a row of the block move their j point to row
// 64 + slot, so the next block can take rows [0, 64).  A slot keeps its pair
// until a drain takes it (the queue is binned from its end), so a row
// 64 + q always belongs to the pair in slot q, and the copies (rows below
// 64 to rows from 64) never overlap.
template <int LOS>
__device__ __forceinline__ void carry_j(WaveState& w, int lane) {
    if (LOS != 1 || w.qtail == 0) return;
    wave_sync_lds();
    if (uint32_t(lane) < w.qtail) {
        const uint32_t jl = uint32_t(__float_as_int(w.qa[lane].w));
        if (jl < 64u) {
            const uint32_t to = 64u + uint32_t(lane);
            const lds_f32_t* src = lds_f32_at(w.jbyte + jl * 12u);
            lds_f32_t* dst = lds_f32_at(w.jbyte + to * 12u);
            const float a = src[0], b = src[1], c = src[2];
            dst[0] = a;
            dst[1] = b;
            dst[2] = c;
            w.qa[lane].w = __int_as_float(int(to));
        }
    }
    wave_sync_lds();
}

// Four i points (ib + k .. ib + k + 3, i cell frame, read with wave-uniform
// scalar loads) against the j block held one point per lane.  TAIL: some of
// the four lie past the chunk (still inside the padded point array); their
// tests are computed and their ballots cleared.  jw: this lane's j point as
// queued for the midpoint line of sight (its row of the j table, as float
// bits).
template <int LOS, bool UNIFORM, bool HAS_EMIN, bool SELF, bool TAIL, bool H16>
__device__ __forceinline__ uint32_t sweep_group(WaveState& w, int lane, float xj, float yj, float zj,
                                                int jrel, const float* __restrict__ q, float jw, int k,
                                                int n_i, uint32_t qt, const PcParams& p,
                                                const ExactTab* __restrict__ xt) {
    float a[12];
#pragma unroll
    for (int t = 0; t < 12; t++) a[t] = q[t];
    Cand c[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        c[u] = test_pair<LOS, HAS_EMIN>(xj, yj, zj, a[3 * u], a[3 * u + 1], a[3 * u + 2], p);
        if (SELF) c[u].acc = c[u].acc && (jrel > k + u);
    }
    // ballots before any branch keep the four distance chains together; one
    // ballot per compare (each is the compare's own lane mask), combined on
    // the scalar unit
    unsigned long long bal[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        unsigned long long b = __builtin_amdgcn_ballot_w64(c[u].d2 < p.emax2_hi);
        if (LOS == 2) b &= __builtin_amdgcn_ballot_w64(fabsf(c[u].dz) < p.pimax_f);
        if (HAS_EMIN) b &= __builtin_amdgcn_ballot_w64(c[u].d2 >= p.emin2_lo);
        if (SELF) b &= __builtin_amdgcn_ballot_w64(jrel > k + u);
        if (TAIL && k + u >= n_i) b = 0;
        bal[u] = b;
    }
#pragma unroll
    for (int u = 0; u < 4; u++)
        qt = push<LOS, UNIFORM, HAS_EMIN, H16>(w, lane, c[u], jw, bal[u], qt, p, xt);
    return qt;
}

// Test the n_i points of the i chunk (ib .. ib + n_i - 1) against the j block.
// The chunk's 768 bytes stay in the scalar cache while every j block of the
// chunk sweeps them.
template <int LOS, bool UNIFORM, bool HAS_EMIN, bool SELF, bool H16>
__device__ __forceinline__ void sweep_block(WaveState& w, int lane, float xj, float yj, float zj, int jrel,
                                            float jw, const float* __restrict__ pts, int64_t ib, int n_i,
                                            const PcParams& p, const ExactTab* __restrict__ xt) {
    // the group's first point, advanced 12 floats a group (a running scalar
    // pointer, where the index arithmetic took a 64-bit multiply per group)
    const float* q = pts + 3 * uniform64(ib);
    uint32_t qt = w.qtail;
    int k = 0;
    for (; k + 4 <= n_i; k += 4, q += 12)
        qt = sweep_group<LOS, UNIFORM, HAS_EMIN, SELF, false, H16>(w, lane, xj, yj, zj, jrel, q, jw, k, n_i, qt, p,
                                                              xt);
    if (k < n_i)
        qt = sweep_group<LOS, UNIFORM, HAS_EMIN, SELF, true, H16>(w, lane, xj, yj, zj, jrel, q, jw, k, n_i, qt, p, xt);
    w.qtail = qt;
}

// Six waves per SIMD (80 VGPRs): latency hiding pays more than the few
// registers this spills outside the inner loops.
template <int LOS, bool UNIFORM, bool HAS_EMIN, bool H16>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) void k_pair_count(
    const float* __restrict__ pts, const int64_t* __restrict__ cs,
    const int2* __restrict__ tasks, const int32_t* __restrict__ order, const int4* __restrict__ sten,
    const ExactTab* __restrict__ xt, const int32_t* __restrict__ otab, unsigned long long* __restrict__ counts,
    unsigned long long* __restrict__ stats, unsigned* __restrict__ queue, PcParams p) {
    // LDS: [histogram, hist_stride words][control, 4 words][one queue of kQ
    // entries per wave][one integer-rule queue per wave: kX, kX16 or kXm
    // entries][midpoint: one j table of kJ 12-byte rows per wave]
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwave = blockDim.x >> 6;
    unsigned* ctl = reinterpret_cast<unsigned*>(smem) + p.hist_stride;
    WaveState w;
    w.hist = reinterpret_cast<unsigned*>(smem);
    w.pj = pts;
    w.b0 = 0;
    const uint32_t qbyte = uint32_t(p.queue_byte0) + uint32_t(wid) * uint32_t(kQ * 16);
    w.qa = reinterpret_cast<float4*>(smem + qbyte);
    // the queue's first slot in a vector register (the append's lane count
    // adds it); the midpoint kernel, which holds the most scalars, also keeps
    // its binning constants there; the other kernels keep them scalar, where
    // their vector registers are the scarcer
    w.qbyte = vreg(qbyte >> 4);
    if (LOS == 1) {
        w.bc.mu_shift = vreg(p.mu_shift);
        w.bc.ok_m = vreg(p.ok_m);
        w.bc.nmu4 = vreg(p.nmu4);
    }
    constexpr int xbytes = kx_bytes(LOS, H16);
    w.xa = reinterpret_cast<float4*>(smem + p.queue_byte0 + nwave * kQ * 16 + wid * xbytes);
    w.xj = w.xa + kXm;
    {
        const uint32_t jbyte = uint32_t(p.queue_byte0) + uint32_t(nwave) * uint32_t(kQ * 16 + xbytes) +
                               uint32_t(wid) * uint32_t(kJ * 12);
        w.jbyte = LOS == 1 ? vreg(jbyte) : jbyte;
    }
    w.xn = 0;
    w.qtail = 0;
    w.since_flush = 0;
    w.n_cand = 0;
    w.n_exact = w.n_flush = w.n_wflush = 0;
    for (int b = threadIdx.x; b < p.hist_stride; b += blockDim.x) w.hist[b] = H16 ? p.h16_init : 0u;
    if (H16) {
        w.nbins = p.nbins;
        w.dst = counts;
    }

    // work items are taken by the whole block (thread 0 pops, the others read
    // the item from LDS), so the block's waves always count the same task
    int xq = int(blockIdx.x % kXcd);
    int exhausted = 0;
    int cur_task = -1;
    for (;;) {
        __syncthreads();  // the previous item is done everywhere; ctl is free
        if (threadIdx.x == 0) {
            unsigned it = 0xFFFFFFFFu;
            while (exhausted < kXcd) {
                const unsigned v = p.qstart[xq] + atomicAdd(&queue[xq], 1u);
                if (v < p.qstart[xq + 1]) {
                    it = v;
                    break;
                }
                ++exhausted;
                xq = (xq + 1) % kXcd;
            }
            ctl[0] = it;
        }
        __syncthreads();
        const unsigned item = __builtin_amdgcn_readfirstlane(ctl[0]);
        if (item == 0xFFFFFFFFu) break;
        int task, g;
        if (p.single_task >= 0) {
            task = p.single_task;
            g = int(item);
        } else {
            task = order[item / unsigned(p.items_per_task)];
            g = int(item % unsigned(p.items_per_task));
        }
        task = __builtin_amdgcn_readfirstlane(task);
        if (task != cur_task) {
            if (cur_task >= 0) {
                drain_all<LOS, UNIFORM, HAS_EMIN, H16>(w, lane, p, xt);
                block_flush<H16>(w.hist, p.nbins, p.h16_init, counts + int64_t(cur_task) * p.nbins);
                if (threadIdx.x == 0) w.n_flush++;
            }
            w.since_flush = 0;
            cur_task = task;
            if (H16) w.dst = counts + int64_t(task) * p.nbins;
            // the task's j catalogue: points are gathered by their byte
            // offset from its first point (catalogues hold fewer than 2^28
            // points)
            const int64_t cat0 = int64_t(tasks[task].y) * p.ncell * p.nsub;
            const int64_t b0 = uniform64(cs[cat0]);
            w.b0 = b0;
            w.pj = pts + 3 * b0;
        }
        unsigned long long* const dst = counts + int64_t(task) * p.nbins;
        const int2 tk = tasks[task];
        const bool autop = tk.x == tk.y;
        const int64_t abase = int64_t(tk.x) * p.ncell, bbase = int64_t(tk.y) * p.ncell;
        const int c0 = g * p.cells_per_item;
        const int c1 = min(c0 + p.cells_per_item, int(p.ncell));
        const int ns = autop ? p.nhalf : p.nfull;
        const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
        const int32_t* ox = otab;
        const int32_t* oy = otab + nx;
        const int32_t* oz = otab + nx + ny;
        const int box = int(p.box);
        const int nsub = p.nsub, sub = p.sub;
        // this lane's sub-cell (lanes >= nsub test nothing)
        const int slx = lane % sub, sly = (lane / sub) % sub, slz = lane / (sub * sub);
        // what a queued pair holds in place of d2 (midpoint): its j point's
        // row in the j table, this lane
        const float jrow = __int_as_float(lane);
        for (int c = c0; c < c1; ++c) {
            const int64_t ia0 = cs[(abase + c) * nsub], ia1 = cs[(abase + c + 1) * nsub];
            if (ia0 == ia1) continue;
            const int cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
            const int oix = ox[cx], oiy = oy[cy], oiz = oz[cz];
            for (int64_t ib = ia0; ib < ia1; ib += p.chunk) {
                // i chunk: points ib .. ib + n_i - 1 of the i cell; its bounding
                // box from one point per lane per slice of 64
                const int n_i = int(min(int64_t(p.chunk), ia1 - ib));
                float blx = 3e38f, bly = 3e38f, blz = 3e38f;
                float bhx = -3e38f, bhy = -3e38f, bhz = -3e38f;
                for (int s0 = 0; s0 < n_i; s0 += 64) {
                    if (lane < n_i - s0) {
                        const int64_t gi = ib + s0 + lane;
                        const float xi = pts[3 * gi], yi = pts[3 * gi + 1], zi = pts[3 * gi + 2];
                        blx = fminf(blx, xi);
                        bly = fminf(bly, yi);
                        blz = fminf(blz, zi);
                        bhx = fmaxf(bhx, xi);
                        bhy = fmaxf(bhy, yi);
                        bhz = fmaxf(bhz, zi);
                    }
                }
                for (int o = 32; o > 0; o >>= 1) {
                    blx = fminf(blx, __shfl_xor(blx, o));
                    bly = fminf(bly, __shfl_xor(bly, o));
                    blz = fminf(blz, __shfl_xor(blz, o));
                    bhx = fmaxf(bhx, __shfl_xor(bhx, o));
                    bhy = fmaxf(bhy, __shfl_xor(bhy, o));
                    bhz = fmaxf(bhz, __shfl_xor(bhz, o));
                }
                // j points gathered into blocks of 64 (one per lane) across runs
                // of kept sub-cells and stencil offsets
                // the wave's share of the bound on every bin, and the count of
                // candidate tests, before nfill j points meet the chunk
                auto account = [&](int nfill) {
                    const uint64_t nc = uint64_t(n_i) * uint64_t(nfill);
                    w.n_cand += nc;
                    // (nc <= 2^14; the sum is taken in 64 bits, so a limit of
                    // 2^32 - 1 cannot wrap)
                    if (uint64_t(w.since_flush) + nc >= uint64_t(p.wave_limit))
                        wave_flush<LOS, UNIFORM, HAS_EMIN, H16>(w, lane, p, xt, dst);
                    w.since_flush += uint32_t(nc);
                };
                // Auto pairs inside the i cell (i < j): its points after the
                // chunk start, in blocks of 64 swept directly by the block's
                // first wave, each lane's j index relative to the chunk start
                // (i indices within the chunk are below 256).
                if (autop && wid == 0) {
                    for (int64_t jb = ib + 1; jb < ia1; jb += 64) {
                        const int n = int(min(ia1 - jb, int64_t(64)));
                        const int32_t jo = int32_t(jb - w.b0);
                        const int32_t io = int32_t(jb - ib);
                        float x = -1e18f, y = -1e18f, z = -1e18f;
                        int rel = INT_MAX;
                        if (lane < n) {
                            const uint32_t off = uint32_t(lane + jo) * 12u;
                            const float* q =
                                reinterpret_cast<const float*>(reinterpret_cast<const char*>(w.pj) + off);
                            x = q[0];
                            y = q[1];
                            z = q[2];
                            rel = lane + io;
                        }
                        account(n);
                        stage_j<LOS>(w, lane, x, y, z, float(oix), float(oiy), float(oiz));
                        sweep_block<LOS, UNIFORM, HAS_EMIN, true, H16>(w, lane, x, y, z, rel, jrow, pts, ib, n_i, p,
                                                                  xt);
                        carry_j<LOS>(w, lane);
                    }
                }
                // The other j points go through two stages.  Stage 1: gathered
                // points, one per lane in lanes [0, fill): coordinates in the i
                // cell frame.
                float sx = 0.0f, sy = 0.0f, sz = 0.0f;
                int fill = 0;
                // Stage 2: the kept points, lanes [0, kfill): the block that is
                // swept against the chunk.
                float kx = -1e18f, ky = -1e18f, kz = -1e18f;
                int kfill = 0;
                auto process = [&](int nfill) {
                    const bool vj = lane < nfill;
                    // lanes past nfill hold a point far from every i point
                    const float xj = vj ? kx : -1e18f, yj = vj ? ky : -1e18f, zj = vj ? kz : -1e18f;
                    account(nfill);
                    stage_j<LOS>(w, lane, kx, ky, kz, float(oix), float(oiy), float(oiz));
                    sweep_block<LOS, UNIFORM, HAS_EMIN, false, H16>(w, lane, xj, yj, zj, INT_MAX, jrow, pts, ib, n_i,
                                                               p, xt);
                    carry_j<LOS>(w, lane);
                };
                // Move the stage-1 points that lie within r_max of the chunk's
                // box into lanes [kfill, ...) of the kept block (one cross-lane
                // permutation per field) and drop the others: no pair of theirs
                // can be binned.  The coordinates and the box are exact integers
                // in float32, so the gaps are exact, and the rounded squared gap
                // exceeds the true one by at most 3 * 2^-24 (relative), inside
                // the 2^-20 margin of emax2_hi: a point with a binnable pair is
                // always kept.  Returns true when the kept block is full; the
                // kept points past it then wait in stage 1 (they pass the test
                // again), so nothing but the two stages stays live across a sweep.
                auto admit = [&]() -> bool {
                    const bool v = lane < fill;
                    const float gx = fmaxf(fmaxf(blx - sx, sx - bhx), 0.0f);
                    const float gy = fmaxf(fmaxf(bly - sy, sy - bhy), 0.0f);
                    const float gz = fmaxf(fmaxf(blz - sz, sz - bhz), 0.0f);
                    bool keep;
                    if (LOS == 2)
                        keep = v && (fmaf(gx, gx, gy * gy) < p.emax2_hi) && (gz < p.pimax_f);
                    else
                        keep = v && (fmaf(gx, gx, fmaf(gy, gy, gz * gz)) < p.emax2_hi);
                    const unsigned long long km = __builtin_amdgcn_ballot_w64(keep);
                    fill = 0;
                    if (!km) return false;
                    const uint32_t nk = uint32_t(__popcll(km));
                    // a permutation of the 64 lanes: the kept lane of rank r goes
                    // to lane kfill + r, every other lane after them (mod 64)
                    const uint32_t rk =
                        __builtin_amdgcn_mbcnt_hi(uint32_t(km >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(km), 0u));
                    const uint32_t pos = keep ? rk : nk + uint32_t(lane) - rk;
                    const int to = int(((uint32_t(kfill) + pos) & 63u) << 2);
                    const float px = __int_as_float(__builtin_amdgcn_ds_permute(to, __float_as_int(sx)));
                    const float py = __int_as_float(__builtin_amdgcn_ds_permute(to, __float_as_int(sy)));
                    const float pz = __int_as_float(__builtin_amdgcn_ds_permute(to, __float_as_int(sz)));
                    const bool take = lane >= kfill;
                    kx = take ? px : kx;
                    ky = take ? py : ky;
                    kz = take ? pz : kz;
                    const int end = kfill + int(nk);
                    if (end < 64) {
                        kfill = end;
                        return false;
                    }
                    // the points past the full block wrapped to lanes [0, end - 64)
                    sx = px;
                    sy = py;
                    sz = pz;
                    fill = end - 64;
                    kfill = 64;
                    return true;
                };
                // the block's waves share the stencil offsets of the chunk
                for (int s = wid; s < ns; s += nwave) {
                    if (autop && s == 0) continue;  // the i cell itself: above
                    const int4 o = sten[s];
                    int jx = cx + o.x, jy = cy + o.y, jz = cz + o.z;
                    int shx = 0, shy = 0, shz = 0;
                    if (p.periodic) {
                        if (jx < 0) { jx += nx; shx = -box; } else if (jx >= nx) { jx -= nx; shx = box; }
                        if (jy < 0) { jy += ny; shy = -box; } else if (jy >= ny) { jy -= ny; shy = box; }
                        if (jz < 0) { jz += nz; shz = -box; } else if (jz >= nz) { jz -= nz; shz = box; }
                    } else if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) {
                        continue;
                    }
                    const int jc = (jz * ny + jy) * nx + jx;
                    const int64_t sbase = (bbase + jc) * nsub;
                    // origin of the j cell's image in the i cell frame
                    const float dox = float(ox[jx] + shx - oix);
                    const float doy = float(oy[jy] + shy - oiy);
                    const float doz = float(oz[jz] + shz - oiz);
                    // sub-cells farther than r_max from the chunk's box hold no
                    // binned pair; their box is widened by 2 units for the
                    // rounding of the integer cell boundaries
                    unsigned long long runs;
                    {
                        const float lx = dox + float(slx) * p.wf[0] - 2.0f, hx = lx + p.wf[0] + 4.0f;
                        const float ly = doy + float(sly) * p.wf[1] - 2.0f, hy = ly + p.wf[1] + 4.0f;
                        const float lz = doz + float(slz) * p.wf[2] - 2.0f, hz = lz + p.wf[2] + 4.0f;
                        const float gx = fmaxf(0.0f, fmaxf(lx - bhx, blx - hx));
                        const float gy = fmaxf(0.0f, fmaxf(ly - bhy, bly - hy));
                        const float gz = fmaxf(0.0f, fmaxf(lz - bhz, blz - hz));
                        bool keep;
                        if (LOS == 2) {
                            // (r_p, pi): transverse gap against the r_p bound,
                            // line-of-sight gap against pi_max
                            keep = (fmaf(gx, gx, gy * gy) < p.emax2_hi) && (gz < p.pimax_f);
                        } else {
                            keep = fmaf(gx, gx, fmaf(gy, gy, gz * gz)) < p.emax2_hi;
                        }
                        runs = __builtin_amdgcn_ballot_w64((lane < nsub) && keep);
                    }
                    while (runs) {
                        // next run of consecutive kept sub-cells = one range of points
                        const int s0 = __builtin_ctzll(runs);
                        const unsigned long long rest = ~(runs >> s0);
                        const int e = rest ? s0 + __builtin_ctzll(rest) : 64;
                        int64_t jb = uniform64(cs[sbase + s0]);
                        const int64_t je = uniform64(cs[sbase + e]);
                        runs = (e >= 64) ? 0ull : (runs & (~0ull << e));
                        while (jb < je) {
                            // lanes [fill, fill + take) take points jb, jb + 1, ...,
                            // each by its byte offset in the j catalogue
                            const int take = int(min(je - jb, int64_t(64 - fill)));
                            const int32_t jo = int32_t(jb - w.b0) - fill;
                            if (lane >= fill && lane < fill + take) {
                                const uint32_t off = uint32_t(lane + jo) * 12u;
                                const float* q = reinterpret_cast<const float*>(
                                    reinterpret_cast<const char*>(w.pj) + off);
                                sx = q[0] + dox;
                                sy = q[1] + doy;
                                sz = q[2] + doz;
                            }
                            fill += take;
                            jb += take;
                            if (fill == 64 && admit()) {
                                process(64);
                                kfill = 0;
                            }
                        }
                    }
                }
                // the rest of stage 1 (a full kept block leaves fewer than 64
                // points there), then the partial kept block
                while (fill > 0) {
                    if (admit()) {
                        process(64);
                        kfill = 0;
                    }
                }
                if (kfill > 0) process(kfill);
            }
        }
    }
    if (cur_task >= 0) {
        drain_all<LOS, UNIFORM, HAS_EMIN, H16>(w, lane, p, xt);
        block_flush<H16>(w.hist, p.nbins, p.h16_init, counts + int64_t(cur_task) * p.nbins);
        if (threadIdx.x == 0) w.n_flush++;
    }
    if (stats) {
        if (w.n_exact) atomicAdd(&stats[2], (unsigned long long)w.n_exact);
        if (lane == 0) {
            atomicAdd(&stats[0], (unsigned long long)w.n_cand);
            if (w.n_wflush) atomicAdd(&stats[1], (unsigned long long)w.n_wflush);
            if (w.n_flush) atomicAdd(&stats[3], (unsigned long long)w.n_flush);
        }
    }
}

typedef void (*PcKernel)(const float*, const int64_t*, const int2*, const int32_t*, const int4*,
                         const ExactTab*, const int32_t*, unsigned long long*, unsigned long long*, unsigned*,
                         PcParams);

static PcKernel pick_kernel(int los, bool uniform, bool has_emin, bool h16) {
    static const PcKernel tab[2][3][2][2] = {
        {{{k_pair_count<0, false, false, false>, k_pair_count<0, false, true, false>},
          {k_pair_count<0, true, false, false>, k_pair_count<0, true, true, false>}},
         {{k_pair_count<1, false, false, false>, k_pair_count<1, false, true, false>},
          {k_pair_count<1, true, false, false>, k_pair_count<1, true, true, false>}},
         {{k_pair_count<2, false, false, false>, k_pair_count<2, false, true, false>},
          {k_pair_count<2, true, false, false>, k_pair_count<2, true, true, false>}}},
        {{{k_pair_count<0, false, false, true>, k_pair_count<0, false, true, true>},
          {k_pair_count<0, true, false, true>, k_pair_count<0, true, true, true>}},
         {{k_pair_count<1, false, false, true>, k_pair_count<1, false, true, true>},
          {k_pair_count<1, true, false, true>, k_pair_count<1, true, true, true>}},
         {{k_pair_count<2, false, false, true>, k_pair_count<2, false, true, true>},
          {k_pair_count<2, true, false, true>, k_pair_count<2, true, true, true>}}},
    };
    return tab[h16 ? 1 : 0][los][uniform ? 1 : 0][has_emin ? 1 : 0];
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
    size_t off_tasks, off_order, off_sten, off_e2, off_otab, off_queue;
    int n_queue;
};

static float f32_up(double v) {  // smallest float >= v
    float f = float(v);
    if (double(f) < v) f = std::nextafter(f, INFINITY);
    return f;
}

static float f32_down(double v) {  // largest float <= v
    float f = float(v);
    if (double(f) > v) f = std::nextafter(f, -INFINITY);
    return f;
}

static lc_status make_plan(DeviceCtx* ctx, const lc_cells* cells, const lc_task* tasks, int32_t n_tasks,
                           const lc_binning* b, int32_t mode, const lc_tuning* tune, Plan& pl) {
    const GridGeom& g = cells->g;
    const int n_r = b->n_r, n_mu = b->n_mu;
    PcParams& p = pl.p;
    std::memset(&p, 0, sizeof p);
    for (int a = 0; a < 3; a++) {
        p.n[a] = g.n[a];
        p.lo[a] = g.lo[a];
        p.ext[a] = g.ext[a];
    }
    p.periodic = g.periodic;
    p.box = g.box;
    p.ncell = g.ncell;
    p.sub = g.sub;
    p.nsub = g.nsub;
    for (int a = 0; a < 3; a++) p.wf[a] = float(double(g.ext[a]) / (double(g.n[a]) * g.sub));
    std::vector<int4> sten;
    const int64_t rmax = b->r_edges[n_r];
    const bool rppi = b->los == LC_LOS_RPPI;
    p.nhalf = build_stencil(g, rmax, rppi ? int64_t(b->pi_max) : 0, sten);
    p.nfull = int(sten.size());
    // relative coordinates and the cell-origin offsets used in float32 must
    // stay below 2^24 in magnitude (exact integers)
    for (int a = 0; a < 3; a++) {
        int kmax = 0;
        for (const int4& o : sten) kmax = std::max(kmax, std::abs(a == 0 ? o.x : a == 1 ? o.y : o.z));
        const int64_t w = (g.ext[a] + g.n[a] - 1) / g.n[a];
        if ((int64_t(kmax) + 1) * w >= (int64_t(1) << 24))
            return fail(LC_ERR_RANGE, "cells of %lld units with a stencil of %d cells exceed the float32 "
                                      "coordinate range; build the mesh with smaller cells",
                        (long long)w, kmax);
    }
    int cpi = tune && tune->cells_per_item > 0 ? tune->cells_per_item : 0;
    if (cpi <= 0) {
        // batched: one row of cells per item (neighbouring items share their j
        // cells); one launch per task: single cells, to spread a task widest
        cpi = (mode & LC_PER_TASK) ? 1 : std::max(1, g.n[0]);
    }
    cpi = int(std::min<int64_t>(cpi, g.ncell));
    p.cells_per_item = cpi;
    p.items_per_task = int((g.ncell + cpi - 1) / cpi);
    p.n_r = n_r;
    p.n_mu = n_mu;
    p.nbins = n_r * n_mu;
    const bool mid = b->los == LC_LOS_MID;
    const int max_chunk = 256;
    // default: a whole cell per gather of its j points (fewer, larger chunks
    // cost a few more candidate tests but gather j points less often)
    const int chunk = tune && tune->chunk > 0 ? tune->chunk : max_chunk;
    if (chunk > max_chunk || chunk % 4 != 0)
        return fail(LC_ERR_INVALID, "chunk = %d, must be a multiple of 4 in [4, %d]", chunk, max_chunk);
    p.chunk = chunk;
    const int64_t e0 = b->r_edges[0];
    const int64_t de = int64_t(b->r_edges[1]) - b->r_edges[0];
    bool uniform = true;
    for (int k = 0; k <= n_r; k++)
        if (int64_t(b->r_edges[k]) != e0 + int64_t(k) * de) uniform = false;
    const int64_t emin2 = e0 * e0, emax2 = rmax * rmax;
    // phase A acceptance: the float32 squared distance is within 3 * 2^-24
    // (relative) of the exact one, inside the 2^-20 margins used here
    p.emax2_hi = f32_up(double(emax2) * (1.0 + std::ldexp(1.0, -20)));
    p.emin2_lo = f32_down(double(emin2) * (1.0 - std::ldexp(1.0, -20)));
    p.inv_drf = float(1.0 / double(de));
    // (r_p, pi): the pi estimate is |s_z| n_pi / pi_max
    p.nmuf = rppi ? float(double(n_mu) / double(b->pi_max)) : float(n_mu);
    p.pimax_f = rppi ? float(b->pi_max) : 0.0f;
    // Float32 error bounds in units of u = 2^-24 (relative error per rounding;
    // v_rsq_f32 is within 1 ulp = 2u):
    //   d2 (float32 sum of exact squares): 3u
    //   mu estimate |s_z| rsq(d2) n_mu - eps_m: 1.5u (from d2) + 2u + a product
    //     and an fma 2u -> 5.5u n_mu absolute; midpoint, all in float32:
    //     l = fma(2, x_j, -s) rounds once (u relative per component), so
    //     |fl(s.l) - s.l| <= (3u + u)|s||l| (three roundings of the dot
    //     product, Cauchy-Schwarz) = 4u of mu; q = fl(l.l) within 5u, so
    //     rsq(q) within 2.5u + 2u; rsq(d2) within 3.5u; two products 2u:
    //     |p| rsq(d2) rsq(q) = mu +- (4u + 10u mu) -> 14u, plus the fma u,
    //     so 15u n_mu, taken as 16u n_mu; (r_p, pi): the exact |s_z|
    //     times a rounded n_pi / pi_max in one fma -> 2u n_pi (r_p^2, a sum of
    //     two exact squares, is within the 3u of d2)
    //   r estimate d2 rsq(d2): 1.5u + 2u + 1u = 4.5u of r; t = r/de - (e0/de +
    //     eps_r) by one fma with rounded 1/de and a rounded shift ->
    //     u (5.5 r_max + e0)/de + u (n_r + 1)
    // The margins are 4x these bounds; pairs closer to an edge take the
    // integer rule.
    const double u = std::ldexp(1.0, -24);
    const double em = (mid ? 16.0 : 5.5) * u * n_mu;
    const float eps_m = f32_up(std::max(4.0 * em, std::ldexp(1.0, -22)));
    const double er = u * ((5.5 * double(rmax) + double(e0)) / double(de) + double(n_r) + 1.0);
    // plus the distance of an accepted pair outside [e_0, e_n) from the edge:
    // phase A accepts d2 < e_n^2 (1 + 2^-20) and d2 >= e_0^2 (1 - 2^-20), i.e.
    // |r - edge| < 2^-20 edge, which is at most 2^-20 r_max / de in units of t
    const double margin_t = std::ldexp(double(rmax) / double(de), -20);
    const float eps_r = f32_up(std::max(4.0 * er + 2.0 * margin_t, std::ldexp(1.0, -22)));
    p.mu_shift = eps_m;
    p.ok_m = f32_down(1.0 - 2.0 * double(eps_m));
    p.r_shift = float(double(e0) / double(de) + double(eps_r));
    p.ok_r = f32_down(1.0 - 2.0 * double(eps_r));
    // LC_FORCE_EXACT: no fraction is below a negative bound, so every pair
    // takes the integer rule
    if (mode & LC_FORCE_EXACT) p.ok_r = -1.0f;
    const bool has_emin = e0 > 0;
    pl.mode = mode;
    pl.n_tasks = n_tasks;
    // Histogram layout: 32-bit bins, or two 16-bit bins per word (H16) with
    // exact wrap accounting and a shorter integer-rule queue: half the LDS
    // for a large histogram, so more waves fit on a CU.
    const int los_k = mid ? 1 : rppi ? 2 : 0;
    const int hist_bits = tune ? tune->hist_bits : 0;
    if (hist_bits != 0 && hist_bits != 16 && hist_bits != 32)
        return fail(LC_ERR_INVALID, "hist_bits = %d, must be 0, 16 or 32", hist_bits);
    struct Shape {
        bool h16;
        PcKernel kern;
        int32_t hist_stride, queue_byte0;
        int wpb, occ;
    };
    auto lds_of = [&](const Shape& sh, int w) {
        return size_t(sh.queue_byte0) +
               size_t(w) * (kQ * 16 + kx_bytes(mid ? 1 : 0, sh.h16) + (mid ? kJ * 12 : 0));
    };
    auto shape_for = [&](bool h16, Shape& sh) -> lc_status {
        sh.h16 = h16;
        sh.kern = pick_kernel(los_k, uniform, has_emin, h16);
        // + the discard slot
        sh.hist_stride = h16 ? ((p.nbins + 1 + 1) / 2 + 3) & ~3 : (p.nbins + 1 + 3) & ~3;
        sh.queue_byte0 = (sh.hist_stride * 4 + 16 + 15) & ~15;
        sh.wpb = sh.occ = 0;
        {
            // the histogram is addressed from LDS address 0 (lds_u32_at): the
            // dynamic block must not follow any static LDS
            hipFuncAttributes fa;
            LC_TRY_HIP(hipFuncGetAttributes(&fa, (const void*)sh.kern));
            if (fa.sharedSizeBytes != 0)
                return fail(LC_ERR_HIP, "pair-count kernel holds %zu bytes of static LDS",
                            size_t(fa.sharedSizeBytes));
        }
        if (lds_of(sh, 1) > ctx->max_lds_block)
            return fail(LC_ERR_INVALID, "histogram of %d bins does not fit in LDS", p.nbins);
        if (lds_of(sh, 16) > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)sh.kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               int(std::min(lds_of(sh, 16), ctx->max_lds_block)));
            if (e != hipSuccess) return fail(LC_ERR_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
        }
        int& wpb = sh.wpb;
        int& occ = sh.occ;
        if (tune && tune->waves_per_block > 0) {
            wpb = tune->waves_per_block;
            if (wpb != 1 && wpb != 2 && wpb != 4 && wpb != 8 && wpb != 12 && wpb != 16)
                return fail(LC_ERR_INVALID, "waves_per_block = %d, must be 1, 2, 4, 8, 12 or 16", wpb);
            while (wpb > 1 && lds_of(sh, wpb) > ctx->max_lds_block) wpb >>= 1;
            LC_TRY_HIP(
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)sh.kern, wpb * 64, lds_of(sh, wpb)));
        } else if (mode & LC_PER_TASK) {
            // one task per launch has few items: the largest blocks finish each
            // item soonest, which shortens the launch's tail (1000 c2 mocks: 2.85 s
            // with 16 waves per block against 4.30 s with 4)
            wpb = 16;
            while (wpb > 1 && lds_of(sh, wpb) > ctx->max_lds_block) wpb >>= 1;
            LC_TRY_HIP(
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)sh.kern, wpb * 64, lds_of(sh, wpb)));
        } else {
            // the block shape that keeps the most waves resident per CU, the
            // smallest on a tie: a small histogram leaves room for several
            // 4-wave blocks, a large one for a single block, which then holds
            // more waves sharing its histogram (12-wave blocks with 16-bit
            // bins or the midpoint kernel's j tables: two of them fit where
            // one 16-wave block did)
            int best = -1;
            for (int w : {4, 8, 12, 16}) {
                if (w == 12 && !h16 && !mid) continue;
                if (lds_of(sh, w) > ctx->max_lds_block) continue;
                int o = 0;
                LC_TRY_HIP(
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, (const void*)sh.kern, w * 64, lds_of(sh, w)));
                if (o * w > best) {
                    best = o * w;
                    wpb = w;
                    occ = o;
                }
            }
            if (wpb == 0) {
                wpb = 4;
                while (wpb > 1 && lds_of(sh, wpb) > ctx->max_lds_block) wpb >>= 1;
                LC_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)sh.kern, wpb * 64,
                                                                        lds_of(sh, wpb)));
            }
        }
        return LC_OK;
    };
    Shape shape;
    LC_TRY(shape_for(hist_bits == 16, shape));
    if (hist_bits == 0 && !(mode & LC_PER_TASK)) {
        // 16-bit bins only where the 32-bit histogram keeps waves off the CU
        // (a 32-bit histogram costs nothing per pair; the 16-bit one costs
        // the wrap check)
        Shape s16;
        LC_TRY(shape_for(true, s16));
        if (s16.wpb * s16.occ > shape.wpb * shape.occ) shape = s16;
    }
    const bool h16 = shape.h16;
    pl.kern = shape.kern;
    p.hist_stride = shape.hist_stride;
    p.queue_byte0 = shape.queue_byte0;
    p.nmu4 = uint32_t((h16 ? 2 : 4) * n_mu);
    // wrap test: every 16-bit bin starts 16 counts below its wrap
    p.h16_init = (h16 && tune && tune->wrap_test) ? 0xFFF0FFF0u : 0u;
    int wpb = shape.wpb, occ = shape.occ;
    pl.threads = wpb * 64;
    pl.lds = lds_of(shape, wpb);
    // each wave's share of the 2^32 bound on a 32-bit bin (16-bit bins are
    // corrected at every wrap and need no bound); a smaller flush_limit
    // (testing) makes waves take the overflow guard early
    p.wave_limit = h16 ? 0xFFFFFFFFu : uint32_t(0xFFFFFFFFu / unsigned(wpb));
    if (tune && tune->flush_limit > 0) p.wave_limit = std::min(p.wave_limit, uint32_t(tune->flush_limit));
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
        return fail(LC_ERR_OVERFLOW, "%lld work items exceed the 31-bit queue", (long long)n_items);
    const bool per_task = (mode & LC_PER_TASK) != 0;
    const int qorder = tune ? tune->queue_order : LC_QUEUE_XCD_RANGES;
    if (qorder != LC_QUEUE_XCD_RANGES && qorder != LC_QUEUE_XCD_DEALT && qorder != LC_QUEUE_SHARED)
        return fail(LC_ERR_INVALID, "queue_order = %d is not LC_QUEUE_XCD_RANGES, _DEALT or _SHARED", qorder);
    p.single_task = -1;
    if (per_task) {
        // one queue holds the task's items; the other queues start empty
        p.qstart[0] = 0;
        for (int x = 1; x <= kXcd; x++) p.qstart[x] = uint32_t(p.items_per_task);
        pl.n_queue = n_tasks * kXcd;
        pl.task_blocks.resize(n_tasks);
        for (int t = 0; t < n_tasks; t++)
            pl.task_blocks[t] = int(std::max<int64_t>(1, std::min<int64_t>(p.items_per_task, pl.blocks)));
    } else if (qorder == LC_QUEUE_XCD_RANGES) {
        // split the ordered tasks into kXcd contiguous ranges of equal cost;
        // blocks of XCD x start on range x and move on when it is empty
        double total = 0;
        for (int t = 0; t < n_tasks; t++) total += cost[t];
        p.qstart[0] = 0;
        double acc = 0;
        int x = 1;
        for (int s = 0; s < n_tasks && x < kXcd; s++) {
            acc += cost[order[s]];
            while (x < kXcd && acc >= total * x / kXcd) p.qstart[x++] = uint32_t(int64_t(s + 1) * p.items_per_task);
        }
        for (; x <= kXcd; x++) p.qstart[x] = uint32_t(n_items);
        pl.n_queue = kXcd;
    } else if (qorder == LC_QUEUE_XCD_DEALT) {
        // task s of the cost order goes to queue s mod kXcd: every queue
        // starts with large tasks and holds tasks of every size
        std::vector<int32_t> dealt;
        dealt.reserve(n_tasks);
        p.qstart[0] = 0;
        for (int x = 0; x < kXcd; x++) {
            for (int s = x; s < n_tasks; s += kXcd) dealt.push_back(order[s]);
            p.qstart[x + 1] = uint32_t(int64_t(dealt.size()) * p.items_per_task);
        }
        order.swap(dealt);
        pl.n_queue = kXcd;
    } else {
        // one queue in cost order: blocks of the other XCDs find theirs empty
        // and move on to it
        p.qstart[0] = 0;
        for (int x = 1; x <= kXcd; x++) p.qstart[x] = uint32_t(n_items);
        pl.n_queue = kXcd;
    }
    // staged block: tasks, order, stencil, squared edges, zeroed queue counters
    std::vector<int64_t> e2(n_r + 1);
    for (int k = 0; k <= n_r; k++) e2[k] = int64_t(b->r_edges[k]) * int64_t(b->r_edges[k]);
    std::vector<unsigned char> xtab(offsetof(ExactTab, e2) + sizeof(int64_t) * e2.size());
    {
        ExactTab head;
        std::memset(&head, 0, sizeof head);
        head.emin2 = emin2;
        head.emax2 = emax2;
        head.e0 = e0;
        head.de = de;
        head.n_r = n_r;
        head.n_mu = n_mu;
        head.discard = p.nbins;
        head.pi_max = rppi ? int64_t(b->pi_max) : 0;
        std::memcpy(xtab.data(), &head, offsetof(ExactTab, e2));
        std::memcpy(xtab.data() + offsetof(ExactTab, e2), e2.data(), sizeof(int64_t) * e2.size());
    }
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
    pl.off_e2 = put(xtab.data(), xtab.size());
    // integer origin of every cell index along x, y and z
    std::vector<int32_t> ot;
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < g.n[a]; c++) ot.push_back(int32_t(cell_origin(c, g.lo[a], g.ext[a], g.n[a])));
    pl.off_otab = put(ot.data(), sizeof(int32_t) * ot.size());
    pl.off_queue = put(qz.data(), sizeof(unsigned) * qz.size());
    return LC_OK;
}

static void launch_plan(const Plan& pl, const lc_cells* cells, unsigned char* dev, uint64_t* counts,
                        uint64_t* stats, hipStream_t s) {
    const int2* d_tasks = reinterpret_cast<const int2*>(dev + pl.off_tasks);
    const int32_t* d_order = reinterpret_cast<const int32_t*>(dev + pl.off_order);
    const int4* d_sten = reinterpret_cast<const int4*>(dev + pl.off_sten);
    const ExactTab* d_e2 = reinterpret_cast<const ExactTab*>(dev + pl.off_e2);
    const int32_t* d_ot = reinterpret_cast<const int32_t*>(dev + pl.off_otab);
    unsigned* d_q = reinterpret_cast<unsigned*>(dev + pl.off_queue);
    auto* c = reinterpret_cast<unsigned long long*>(counts);
    auto* st = reinterpret_cast<unsigned long long*>(stats);
    if (pl.mode & LC_PER_TASK) {
        PcParams p = pl.p;
        for (int t = 0; t < pl.n_tasks; t++) {
            p.single_task = t;
            hipLaunchKernelGGL(pl.kern, dim3(pl.task_blocks[t]), dim3(pl.threads), pl.lds, s, cells->pts,
                               cells->cs, d_tasks, d_order, d_sten, d_e2, d_ot, c, st, d_q + kXcd * t, p);
        }
    } else {
        hipLaunchKernelGGL(pl.kern, dim3(pl.blocks), dim3(pl.threads), pl.lds, s, cells->pts, cells->cs, d_tasks,
                           d_order, d_sten, d_e2, d_ot, c, st, d_q, pl.p);
    }
}

// Graph cache: captured launch sequences keyed by everything they bake in,
// the mesh's device buffers included.  lc_free_cells drops the entries of
// the mesh it frees (forget_graphs), so no entry outlives its buffers.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    void* dev = nullptr;  // owned copy of the staged block
    const lc_cells* cells = nullptr;
};
static std::mutex g_graph_mu;
static std::map<std::string, GraphEntry> g_graphs;

static std::string graph_key(const Plan& pl, const lc_cells* cells, uint64_t* counts, uint64_t* stats,
                             int device) {
    std::string k;
    auto add = [&](const void* p, size_t n) { k.append(reinterpret_cast<const char*>(p), n); };
    add(&device, sizeof device);
    add(&cells, sizeof cells);
    add(&cells->pts, sizeof cells->pts);
    add(&cells->cs, sizeof cells->cs);
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
        ge.cells = cells;
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

static void destroy_graph(GraphEntry& ge) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    if (ge.graph) (void)hipGraphDestroy(ge.graph);
    if (ge.dev) (void)hipFree(ge.dev);
}

void release_graphs() {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& kv : g_graphs) destroy_graph(kv.second);
    g_graphs.clear();
}

void forget_graphs(const lc_cells* cells) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        if (it->second.cells == cells) {
            destroy_graph(it->second);
            it = g_graphs.erase(it);
        } else {
            ++it;
        }
    }
}

// Argument checks shared by the two pair-count entry points.
static lc_status check_count_args(const lc_cells* cells, const lc_task* tasks, int32_t n_tasks,
                                  const lc_binning* b, uint64_t* counts, int32_t mode) {
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
    return LC_OK;
}

// ---------------------------------------------------------------------------
// allocation-free variant: the staged plan lives in a static device array
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(LC_NOALLOC_PLAN_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device, taken once with that device
// current (host code must never pass the array's name to a kernel: on the
// host it is only a stand-in for the symbol).
static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_ptr;

static lc_status scratch_ptr(int device, unsigned char** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return LC_OK;
    }
    void* ptr = nullptr;
    LC_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(LC_ERR_HIP, "hipGetSymbolAddress returned NULL for the plan array");
    g_scratch_ptr[device] = static_cast<unsigned char*>(ptr);
    *out = static_cast<unsigned char*>(ptr);
    return LC_OK;
}

// The plan reaches the device through kernel arguments, kStageWords words per
// launch: no host staging buffer, no device allocation, and no copy from
// pageable memory.
constexpr int kStageWords = 480;
struct StageArgs {
    uint32_t n;                 // words in this piece
    uint32_t w[kStageWords];
};

__global__ __launch_bounds__(256) void k_stage(uint32_t* __restrict__ dst, StageArgs a) {
    for (uint32_t i = threadIdx.x; i < a.n; i += blockDim.x) dst[i] = a.w[i];
}

}  // namespace lc

using namespace lc;

extern "C" lc_status lc_pair_count_batch(const lc_cells* cells, const lc_task* tasks, int32_t n_tasks,
                                         const lc_binning* b, uint64_t* counts, int32_t mode,
                                         const lc_tuning* tune, uint64_t* stats, void* stream) {
    clear_error();
    LC_TRY(check_count_args(cells, tasks, n_tasks, b, counts, mode));
    if (n_tasks == 0) return LC_OK;
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

extern "C" lc_status lc_pair_count_batch_noalloc(const lc_cells* cells, const lc_task* tasks, int32_t n_tasks,
                                                 const lc_binning* b, uint64_t* counts, int32_t mode,
                                                 const lc_tuning* tune, uint64_t* stats, void* stream) {
    clear_error();
    LC_TRY(check_count_args(cells, tasks, n_tasks, b, counts, mode));
    if (mode & LC_GRAPH)
        return fail(LC_ERR_INVALID, "LC_GRAPH keeps a cached copy of the plan in allocated memory; "
                                    "the allocation-free call takes LC_PERSISTENT or LC_PER_TASK (| LC_FORCE_EXACT)");
    if (n_tasks == 0) return LC_OK;
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    if (ctx->device != cells->device) return fail(LC_ERR_INVALID, "mesh lives on another device");
    Plan pl;
    LC_TRY(make_plan(ctx, cells, tasks, n_tasks, b, mode, tune, pl));
    pl.blob.resize((pl.blob.size() + 3) & ~size_t(3), 0);
    if (pl.blob.size() > kScratchBytes)
        return fail(LC_ERR_OVERFLOW, "the plan of %d tasks takes %zu bytes, more than the %zu bytes of the "
                                     "allocation-free call's static plan array; use lc_pair_count_batch",
                    n_tasks, pl.blob.size(), kScratchBytes);
    unsigned char* dev = nullptr;
    LC_TRY(scratch_ptr(ctx->device, &dev));
    hipStream_t s = (hipStream_t)stream;
    const uint32_t* words = reinterpret_cast<const uint32_t*>(pl.blob.data());
    const size_t n_words = pl.blob.size() / 4;
    StageArgs a;
    for (size_t w0 = 0; w0 < n_words; w0 += kStageWords) {
        a.n = uint32_t(std::min<size_t>(kStageWords, n_words - w0));
        std::memcpy(a.w, words + w0, size_t(a.n) * 4);
        hipLaunchKernelGGL(k_stage, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t*>(dev) + w0, a);
    }
    launch_plan(pl, cells, dev, counts, stats, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LC_ERR_HIP, "pair-count launch failed: %s", hipGetErrorString(e));
    return LC_OK;
}
