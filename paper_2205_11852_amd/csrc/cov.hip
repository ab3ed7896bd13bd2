// Sample covariances over mocks and the linear construction (Sect. 2.2, 2.3),
// plus the positive-definiteness check of the result (Sect. 3).
//
//   mean (float64, two passes)  ->  deviations  ->  Cov_e = D_e^T D_e / (N-1)
//   for the three estimates e = (D,R1), (D,R2), (D,R1uR2)
//   ->  C^a = (Cov_0 + Cov_1)/2, C^b = Cov_2,
//       A = (M_b C^b - M_a C^a)/(M_b - M_a), B = M_a M_b (C^a - C^b)/(M_b - M_a)
//       (Eq. CovAB; 2C^b - C^a and 2 M_a (C^a - C^b) at M_b = 2 M_a),
//       C = A + B/M                                    (float64)
//   ->  Cholesky and eigenvalue extremes of each block of C (float64).
//
// The products D^T D run either in float64 (VALU) or as float32 MFMA
// (v_mfma_f32_32x32x2f32) with float32 accumulation, by default over chunks
// of 256 mocks whose partial sums are added in float64 (LC_ACC32: over all
// mocks in float32).
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "lc_internal.hpp"

namespace lc {

// ---------------------------------------------------------------------------
// mean and deviations
// ---------------------------------------------------------------------------
constexpr int kMeanRows = 64;

// partial[c][j] = sum of xi[n][j] over rows n of chunk c (j < 3P)
__global__ void k_mean_partial(const double* __restrict__ xi, int64_t n_mock, int64_t W3,
                               double* __restrict__ partial) {
    const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (j >= W3) return;
    const int64_t n0 = int64_t(blockIdx.y) * kMeanRows;
    const int64_t n1 = min(n0 + kMeanRows, n_mock);
    double s = 0.0;
    for (int64_t n = n0; n < n1; n++) s += xi[n * W3 + j];
    partial[int64_t(blockIdx.y) * W3 + j] = s;
}

__global__ void k_mean_final(const double* __restrict__ partial, int64_t nchunk, int64_t W3, int64_t n_mock,
                             double* __restrict__ mean) {
    const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (j >= W3) return;
    double s = 0.0;
    for (int64_t c = 0; c < nchunk; c++) s += partial[c * W3 + j];
    mean[j] = s / double(n_mock);
}

// dev64[e][n][p] = xi[n][e][p] - mean[e][p]    (ne estimates per mock; ld = P)
__global__ void k_dev64(const double* __restrict__ xi, const double* __restrict__ mean, int64_t n_mock,
                        int64_t P, int64_t ne, double* __restrict__ dev) {
    const int64_t tot = ne * n_mock * P;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < tot;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t p = t % P;
        const int64_t r = t / P;
        const int64_t n = r % n_mock;
        const int64_t e = r / n_mock;
        dev[t] = xi[n * ne * P + e * P + p] - mean[e * P + p];
    }
}

// dev32[e][n][p] (ld = Ppad, Npad rows, zero padded) = float(xi - mean)
__global__ void k_dev32(const double* __restrict__ xi, const double* __restrict__ mean, int64_t n_mock,
                        int64_t P, int64_t ne, int64_t Npad, int64_t Ppad, float* __restrict__ dev) {
    const int64_t tot = ne * Npad * Ppad;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < tot;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t p = t % Ppad;
        const int64_t r = t / Ppad;
        const int64_t n = r % Npad;
        const int64_t e = r / Npad;
        float v = 0.0f;
        if (n < n_mock && p < P) v = float(xi[n * ne * P + e * P + p] - mean[e * P + p]);
        dev[t] = v;
    }
}

// ---------------------------------------------------------------------------
// SYRK, float64: 64x64 tiles, 16x16 threads with 4x4 outputs each
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tri_tile(int t, int& ti, int& tj) {
    // t enumerates (ti, tj) with tj <= ti
    ti = int((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ti++;
    while (ti * (ti + 1) / 2 > t) ti--;
    tj = t - ti * (ti + 1) / 2;
}

__global__ __launch_bounds__(256) void k_syrk64(const double* __restrict__ dev, int64_t n_mock, int64_t P,
                                                double denom, double* __restrict__ cov) {
    __shared__ double As[16][64 + 1];
    __shared__ double Bs[16][64 + 1];
    const int e = blockIdx.y;
    int ti, tj;
    tri_tile(blockIdx.x, ti, tj);
    const int64_t i0 = int64_t(ti) * 64, j0 = int64_t(tj) * 64;
    const double* D = dev + int64_t(e) * n_mock * P;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4] = {};
    for (int64_t n0 = 0; n0 < n_mock; n0 += 16) {
        for (int q = threadIdx.x; q < 16 * 64; q += 256) {
            const int kk = q >> 6, c = q & 63;
            const int64_t n = n0 + kk;
            As[kk][c] = (n < n_mock && i0 + c < P) ? D[n * P + i0 + c] : 0.0;
            Bs[kk][c] = (n < n_mock && j0 + c < P) ? D[n * P + j0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk++) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                a[r] = As[kk][ty * 4 + r];
                b[r] = Bs[kk][tx * 4 + r];
            }
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int c = 0; c < 4; c++) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
    double* C = cov + int64_t(e) * P * P;
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            const int64_t i = i0 + ty * 4 + r, j = j0 + tx * 4 + c;
            if (i < P && j < P) {
                const double v = acc[r][c] / denom;
                C[i * P + j] = v;
                if (ti != tj) C[j * P + i] = v;
            }
        }
}

// ---------------------------------------------------------------------------
// SYRK, float32 MFMA: 128x128 tile per block, 2x2 waves of 64x64,
// each wave 2x2 blocks of v_mfma_f32_32x32x2f32.
// Operand layout of the 32x32x2 instruction (wave64): lane l supplies
// A[i = l%32][k = l/32] and B[k = l/32][j = l%32]; accumulator register r of
// lane l holds D[i = 8*(r/4) + 4*(l/32) + r%4][j = l%32].
// ---------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMT = 128;    // tile
constexpr int kKT = 32;     // rows per LDS slab
constexpr int kKC = 256;    // rows per float32 accumulation chunk

// kc: rows summed in the float32 accumulators before they are added into
// the float64 ones (a multiple of kKT; Npad or more: float32 throughout)
__global__ __launch_bounds__(256) void k_syrk32(const float* __restrict__ dev, int64_t Npad, int64_t Ppad,
                                                int64_t P, int64_t kc, double denom, double* __restrict__ cov) {
    __shared__ __align__(16) float As[kKT][kMT];
    __shared__ __align__(16) float Bs[kKT][kMT];
    const int e = blockIdx.y;
    int ti, tj;
    tri_tile(blockIdx.x, ti, tj);
    const int64_t i0 = int64_t(ti) * kMT, j0 = int64_t(tj) * kMT;
    const float* D = dev + int64_t(e) * Npad * Ppad;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    const int li = lane & 31, lk = lane >> 5;
    f32x16 acc[2][2];
    double dacc[2][2][16];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            for (int r = 0; r < 16; r++) {
                acc[a][b][r] = 0.0f;
                dacc[a][b][r] = 0.0;
            }
        }
    int64_t since = 0;
    for (int64_t n0 = 0; n0 < Npad; n0 += kKT) {
        // each thread loads 4 float4 of each slab: 32 rows x 128 floats
        for (int q = threadIdx.x; q < kKT * kMT / 4; q += 256) {
            const int kk = q / (kMT / 4), c4 = (q % (kMT / 4)) * 4;
            const float4 va = *reinterpret_cast<const float4*>(D + (n0 + kk) * Ppad + i0 + c4);
            const float4 vb = *reinterpret_cast<const float4*>(D + (n0 + kk) * Ppad + j0 + c4);
            *reinterpret_cast<float4*>(&As[kk][c4]) = va;
            *reinterpret_cast<float4*>(&Bs[kk][c4]) = vb;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kKT; ks += 2) {
            float a0 = As[ks + lk][wr * 64 + li];
            float a1 = As[ks + lk][wr * 64 + 32 + li];
            float b0 = Bs[ks + lk][wc * 64 + li];
            float b1 = Bs[ks + lk][wc * 64 + 32 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
        since += kKT;
        if (since == kc || n0 + kKT >= Npad) {
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 2; b++)
                    for (int r = 0; r < 16; r++) {
                        dacc[a][b][r] += double(acc[a][b][r]);
                        acc[a][b][r] = 0.0f;
                    }
            since = 0;
        }
    }
    double* C = cov + int64_t(e) * P * P;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int r = 0; r < 16; r++) {
                const int64_t i = i0 + wr * 64 + a * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                const int64_t j = j0 + wc * 64 + b * 32 + li;
                if (i < P && j < P) {
                    const double v = dacc[a][b][r] / denom;
                    C[i * P + j] = v;
                    if (ti != tj) C[j * P + i] = v;
                }
            }
}

// ---------------------------------------------------------------------------
// linear construction (float64)
// ---------------------------------------------------------------------------
__global__ void k_combine(const double* __restrict__ cov, int64_t PP, double m_a, double m_b, double M, int m_inf,
                          double* __restrict__ A, double* __restrict__ B, double* __restrict__ C) {
#pragma clang fp contract(off)
    // Eq. CovAB: A = (M_b C^b - M_a C^a)/(M_b - M_a), B = M_a M_b/(M_b - M_a) (C^a - C^b);
    // at M_b = 2 M_a (Eq. LCdef) the forms 2 C^b - C^a and 2 M_a (C^a - C^b)
    // are used as written (the general quotient would round differently
    // unless M_a is a power of two)
    const double dm = m_b - m_a;
    const bool paper = (m_b == 2.0 * m_a);
    const double kb = paper ? 2.0 * m_a : (m_a * m_b) / dm;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < PP;
         t += int64_t(gridDim.x) * blockDim.x) {
        const double ca = 0.5 * (cov[t] + cov[PP + t]);
        const double cb = cov[2 * PP + t];
        const double a = paper ? 2.0 * cb - ca : (m_b * cb - m_a * ca) / dm;
        const double b = kb * (ca - cb);
        A[t] = a;
        B[t] = b;
        C[t] = m_inf ? a : a + b / M;
    }
}

// ---------------------------------------------------------------------------
// Frobenius norms for the float32-vs-float64 report
// ---------------------------------------------------------------------------
__global__ void k_frob(const double* __restrict__ x, const double* __restrict__ y, int64_t n,
                       double* __restrict__ part) {
    __shared__ double sd[256], sy[256];
    double d = 0.0, s = 0.0;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
        const double df = x[t] - y[t];
        d += df * df;
        s += y[t] * y[t];
    }
    sd[threadIdx.x] = d;
    sy[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sd[threadIdx.x] += sd[threadIdx.x + o];
            sy[threadIdx.x] += sy[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sd[0];
        part[2 * blockIdx.x + 1] = sy[0];
    }
}

// ---------------------------------------------------------------------------
// check: copy a diagonal block, Cholesky, Householder tridiagonalisation,
// bisection on the tridiagonal for the extreme eigenvalues and the number of
// negative ones.  Work matrix: n x n row-major, ld = n.
// ---------------------------------------------------------------------------
struct CheckFlags {
    int nan_seen;
    int chol_fail;
};

__global__ void k_copy_block(const double* __restrict__ C, int64_t P, int64_t off, int64_t n,
                             double* __restrict__ W, CheckFlags* fl) {
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n * n; t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = t / n, j = t % n;
        const double v = C[(off + i) * P + off + j];
        W[t] = v;
        if (v != v) fl->nan_seen = 1;
    }
}

__global__ void k_zero_flags(CheckFlags* fl, int n) {
    if (int(threadIdx.x) < n) {
        fl[threadIdx.x].nan_seen = 0;
        fl[threadIdx.x].chol_fail = 0;
    }
}

constexpr int kNB = 32;

// factor the diagonal block [k0, k0+nb) in place (lower triangle)
__global__ void k_potrf_diag(double* __restrict__ W, int64_t n, int64_t k0, int nb, CheckFlags* fl) {
    __shared__ double L[kNB][kNB + 1];
    __shared__ int bad;
    if (fl->chol_fail || fl->nan_seen) return;
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) L[t / nb][t % nb] = W[(k0 + t / nb) * n + k0 + t % nb];
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < nb; j++) {
        if (threadIdx.x == 0) {
            double d = L[j][j];
            for (int q = 0; q < j; q++) d -= L[j][q] * L[j][q];
            if (!(d > 0.0)) bad = 1;
            L[j][j] = bad ? 1.0 : sqrt(d);
        }
        __syncthreads();
        if (bad) break;
        for (int i = j + 1 + threadIdx.x; i < nb; i += blockDim.x) {
            double v = L[i][j];
            for (int q = 0; q < j; q++) v -= L[i][q] * L[j][q];
            L[i][j] = v / L[j][j];
        }
        __syncthreads();
    }
    if (bad) {
        if (threadIdx.x == 0) fl->chol_fail = 1;
        return;
    }
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = t / nb, j = t % nb;
        if (j <= i) W[(k0 + i) * n + k0 + j] = L[i][j];
    }
}

// rows below the diagonal block: L21 = A21 L11^{-T}, one thread per row
__global__ void k_potrf_panel(double* __restrict__ W, int64_t n, int64_t k0, int nb, const CheckFlags* fl) {
    __shared__ double L[kNB][kNB + 1];
    if (fl->chol_fail || fl->nan_seen) return;
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) L[t / nb][t % nb] = W[(k0 + t / nb) * n + k0 + t % nb];
    __syncthreads();
    const int64_t i = k0 + nb + blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double x[kNB];
    for (int j = 0; j < nb; j++) {
        double v = W[i * n + k0 + j];
        for (int q = 0; q < j; q++) v -= x[q] * L[j][q];
        x[j] = v / L[j][j];
    }
    for (int j = 0; j < nb; j++) W[i * n + k0 + j] = x[j];
}

// trailing update of the lower triangle: A22 -= L21 L21^T
__global__ __launch_bounds__(256) void k_potrf_update(double* __restrict__ W, int64_t n, int64_t k0, int nb,
                                                      const CheckFlags* fl) {
    if (fl->chol_fail || fl->nan_seen) return;
    __shared__ double Ai[64][kNB + 1];
    __shared__ double Aj[64][kNB + 1];
    const int64_t base = k0 + nb;
    int ti, tj;
    tri_tile(blockIdx.x, ti, tj);
    const int64_t i0 = base + int64_t(ti) * 64, j0 = base + int64_t(tj) * 64;
    for (int t = threadIdx.x; t < 64 * nb; t += 256) {
        const int r = t / nb, q = t % nb;
        Ai[r][q] = (i0 + r < n) ? W[(i0 + r) * n + k0 + q] : 0.0;
        Aj[r][q] = (j0 + r < n) ? W[(j0 + r) * n + k0 + q] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            const int ir = ty * 4 + r, jc = tx * 4 + c;
            const int64_t i = i0 + ir, j = j0 + jc;
            if (i < n && j < n && j <= i) {
                double s = 0.0;
                for (int q = 0; q < nb; q++) s += Ai[ir][q] * Aj[jc][q];
                W[i * n + j] -= s;
            }
        }
}

// Sum of x over the block (every thread gets the total).
// Wave sums by butterfly shuffles, then one exchange of the per-wave sums
// through `red` (blockDim.x a multiple of 64, at most 1024): two barriers.
__device__ __forceinline__ double block_sum(double x, double* red) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    const int nw = int(blockDim.x >> 6);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < nw; w++) r += red[w];
    __syncthreads();
    return r;
}

// Householder tridiagonalisation of the symmetric block, one launch per
// column k = 0 .. n-3.  Step k reflects row k of the trailing matrix onto
// alpha e1 (v = x - alpha e1, tau = 2 / v.v), forms p = tau A22 v and the
// rank-2 update A22 -= v w^T + w v^T with w = p - K v, K = (tau/2) v.p.
// The launch for column k applies the update of column k-1 as it goes:
// every wave updates its own row of A22(k) while reading it (and writes it
// back), and every block updates row k on the fly from the old row and
// step k-1's v and p, so no block waits for another.  Indices of the
// pending update run over A22(k-1), whose row and column 0 are row and
// column k of W.
struct HhPending {
    const double* v;        // [m + 1] Householder vector of step k-1 (NULL: none pending)
    const double* p;        // [m + 1] tau A v of step k-1
    const double* tau;
    const double* vp_part;  // partial sums of v.p, n1 of them
    int64_t n1;
};

// K of the pending update: the same ordered reduction in every block.
__device__ __forceinline__ double hh_pending_k(const HhPending& q, double* red) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < q.n1; i += blockDim.x) s += q.vp_part[i];
    const double t = block_sum(s, red);
    return q.v ? 0.5 * *q.tau * t : 0.0;
}

// element (i, j) of A22(k-1) with the pending update applied
__device__ __forceinline__ double hh_apply(double a, const HhPending& q, double K, int64_t i, int64_t j) {
    if (!q.v) return a;
    const double wi = q.p[i] - K * q.v[i], wj = q.p[j] - K * q.v[j];
    return a - (q.v[i] * wj + wi * q.v[j]);
}

// The pending update's v and w at index i (zero when none is pending).
struct HhVW {
    double v, w;
};
__device__ __forceinline__ HhVW hh_vw(const HhPending& q, double K, int64_t i) {
    if (!q.v) return HhVW{0.0, 0.0};
    const double v = q.v[i];
    return HhVW{v, q.p[i] - K * v};
}

constexpr int kHhRows = 4;  // rows of A22 per k_hh_column block

// WAVES waves per row: 4 while the trailing matrix is large (more loads in
// flight), 1 once it is small (the launch's fixed cost dominates).  Every
// load that does not depend on the pending update's K (the partial sums
// that give K, this thread's share of row k for the norm, this lane's share
// of its row of A22 with row k beside it, the pending v and p there) is
// issued before the first barrier and held in registers, so a launch waits
// on memory once instead of three times in a row; elements beyond the held
// ones (a trailing matrix wider than the block for the norm, 2 x 256 or
// 4 x 64 per lane for the product, so that two 1024-thread blocks still fit
// on a CU) are read afterwards, the product's two per lane at a time with
// both loads issued before either store (four at a time spill registers).
template <int WAVES>
__global__ __launch_bounds__(64 * kHhRows * WAVES)
__attribute__((amdgpu_waves_per_eu(WAVES == 4 ? 8 : 4))) void k_hh_column(double* __restrict__ W, int64_t n,
                                                                          int64_t k, HhPending q,
                                                   double* __restrict__ v, double* __restrict__ tau,
                                                   double* __restrict__ d, double* __restrict__ e,
                                                   double* __restrict__ pv, double* __restrict__ vp_part) {
    constexpr int NT = 64 * kHhRows * WAVES;   // threads
    constexpr int NPF = 1;                     // row-k elements per thread held for the norm
    constexpr int RPF = WAVES == 4 ? 2 : 4;    // row elements per lane held for the product
    constexpr int64_t RST = 64 * WAVES;        // stride of a lane's row elements
    constexpr int CH = 2;                      // row elements per load group after the held ones
    __shared__ double red[kHhRows * WAVES];
    __shared__ double wsum[kHhRows * WAVES];
    const int64_t m = n - k - 1;
    const bool pend = q.v != nullptr;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = blockIdx.x * int64_t(kHhRows) + wv / WAVES;
    const int64_t jl = int64_t(wv % WAVES) * 64 + lane;
    const bool rowok = r < m;
    // row k beyond the diagonal, old values; its updated value at j is
    // x_j = row[j] - (v_0 w_{j+1} + w_0 v_{j+1}) (pending update, index 0)
    const double* row = W + k * n + k + 1;
    double* ar = W + (k + 1 + (rowok ? r : 0)) * n + k + 1;
    auto pv_at = [&](int64_t i) { return pend ? q.v[i] : 0.0; };
    auto pp_at = [&](int64_t i) { return pend ? q.p[i] : 0.0; };
    // --- loads independent of K
    double kp = 0.0;
    if (pend)
        for (int64_t i = threadIdx.x; i < q.n1; i += NT) kp += q.vp_part[i];
    const double tau_prev = pend ? *q.tau : 0.0;
    const double zv = pv_at(0), zp = pp_at(0);
    const double x0r = row[0], x0v = pv_at(1), x0p = pp_at(1);
    const double yv = rowok ? pv_at(r + 1) : 0.0, yp = rowok ? pp_at(r + 1) : 0.0;
    double nr[NPF], nv[NPF], np[NPF];
#pragma unroll
    for (int t = 0; t < NPF; t++) {
        const int64_t j = threadIdx.x + int64_t(t) * NT;
        const bool ok = j < m;
        nr[t] = ok ? row[j] : 0.0;
        nv[t] = ok ? pv_at(j + 1) : 0.0;
        np[t] = ok ? pp_at(j + 1) : 0.0;
    }
    double ra[RPF], rr[RPF], rv[RPF], rp[RPF];
#pragma unroll
    for (int t = 0; t < RPF; t++) {
        const int64_t j = jl + int64_t(t) * RST;
        const bool ok = rowok && j < m;
        ra[t] = ok ? ar[j] : 0.0;
        rr[t] = ok ? row[j] : 0.0;
        rv[t] = ok ? pv_at(j + 1) : 0.0;
        rp[t] = ok ? pp_at(j + 1) : 0.0;
    }
    // --- K of the pending update: the same ordered reduction in every block
    const double K = pend ? 0.5 * tau_prev * block_sum(kp, red) : 0.0;
    const double zw = zp - K * zv;
    // updated row k at j from the old value and the pending v, p at j + 1
    auto xk = [&](double rj, double vj, double pj) { return pend ? rj - (zv * (pj - K * vj) + zw * vj) : rj; };
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < NPF; t++) {
        const double x = xk(nr[t], nv[t], np[t]);
        s += x * x;
    }
#pragma unroll 2
    for (int64_t j = threadIdx.x + int64_t(NPF) * NT; j < m; j += NT) {
        const double x = xk(row[j], pv_at(j + 1), pp_at(j + 1));
        s += x * x;
    }
    const double norm2 = block_sum(s, red);
    const double x0 = xk(x0r, x0v, x0p);
    const double nrm = sqrt(norm2);
    const double alpha = x0 > 0 ? -nrm : nrm;   // reflect x onto alpha * e1
    const double v0 = x0 - alpha;
    const double vnorm2 = norm2 - x0 * x0 + v0 * v0;
    const bool trivial = !(vnorm2 > 0.0) || (norm2 - x0 * x0) <= 0.0;
    const double t = trivial ? 0.0 : 2.0 / vnorm2;
    if (blockIdx.x == 0) {
        for (int64_t i = threadIdx.x; i < m; i += NT)
            v[i] = trivial ? 0.0 : (i == 0 ? v0 : xk(row[i], pv_at(i + 1), pp_at(i + 1)));
        if (threadIdx.x == 0) {
            // diagonal entry k: the old one less 2 v_0 w_0 of the pending update
            d[k] = pend ? W[k * n + k] - 2.0 * zv * zw : W[k * n + k];
            e[k] = trivial ? x0 : alpha;
            *tau = t;
        }
    }
    // p_r = tau sum_j A22[r][j] v_j, WAVES waves per row (kHhRows rows per
    // block) taking 64 columns in turn; the row is brought up to date
    // (pending update, index r + 1) as it is read and written back
    const double yw = yp - K * yv;
    double acc = 0.0;
    if (rowok) {
#pragma unroll
        for (int tt = 0; tt < RPF; tt++) {
            const int64_t j = jl + int64_t(tt) * RST;
            if (j < m) {
                const double cw = rp[tt] - K * rv[tt];
                double a = ra[tt];
                if (pend) {
                    a = a - (yv * cw + yw * rv[tt]);
                    ar[j] = a;
                }
                acc += a * (j == 0 ? v0 : xk(rr[tt], rv[tt], rp[tt]));
            }
        }
        // the rest in groups of CH elements whose loads are all issued
        // before the group's stores (same order of the sum)
        for (int64_t j0 = jl + int64_t(RPF) * RST; j0 < m; j0 += CH * RST) {
            double ca[CH], cr[CH], cv[CH], cp[CH];
#pragma unroll
            for (int u = 0; u < CH; u++) {
                const int64_t j = j0 + int64_t(u) * RST;
                const bool ok = j < m;
                ca[u] = ok ? ar[j] : 0.0;
                cr[u] = ok ? row[j] : 0.0;
                cv[u] = ok ? pv_at(j + 1) : 0.0;
                cp[u] = ok ? pp_at(j + 1) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CH; u++) {
                const int64_t j = j0 + int64_t(u) * RST;
                if (j < m) {
                    const double cw = cp[u] - K * cv[u];
                    double a = ca[u];
                    if (pend) {
                        a = a - (yv * cw + yw * cv[u]);
                        ar[j] = a;
                    }
                    acc += a * (j == 0 ? v0 : xk(cr[u], cv[u], cp[u]));
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    }
    if (lane == 0) wsum[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int i = 0; i < kHhRows; i++) {
            const int64_t ri = blockIdx.x * int64_t(kHhRows) + i;
            if (ri >= m) break;
            double a = 0.0;
            for (int w = 0; w < WAVES; w++) a += wsum[WAVES * i + w];
            const double p = trivial ? 0.0 : t * a;
            pv[ri] = p;
            b += trivial ? 0.0 : p * (ri == 0 ? v0 : xk(row[ri], pv_at(ri + 1), pp_at(ri + 1)));
        }
        vp_part[blockIdx.x] = b;
    }
}

// The last 2 x 2 block (rows n-2, n-1 = indices 0, 1 of the pending update's
// A22) gives the last diagonal and off-diagonal entries.  One block.
__global__ void k_hh_tail(const double* __restrict__ W, int64_t n, HhPending q, double* __restrict__ d,
                          double* __restrict__ e) {
    __shared__ double red[256];
    const double K = hh_pending_k(q, red);
    if (threadIdx.x != 0) return;
    if (n >= 2) {
        d[n - 2] = hh_apply(W[(n - 2) * n + n - 2], q, K, 0, 0);
        e[n - 2] = hh_apply(W[(n - 1) * n + n - 2], q, K, 1, 0);
    }
    d[n - 1] = hh_apply(W[(n - 1) * n + n - 1], q, K, n >= 2 ? 1 : 0, n >= 2 ? 1 : 0);
}

// number of eigenvalues of the tridiagonal (d, e) below x (Sturm count)
__device__ int sturm_count(const double* d, const double* e, int64_t n, double x, double pivmin) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) c++;
    for (int64_t i = 1; i < n; i++) {
        q = d[i] - x - e[i - 1] * e[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) c++;
    }
    return c;
}

// out: [0] min eig, [1] max eig, [2] count below 0 (as double).  Three
// blocks work at once: block 0 bisects for the smallest eigenvalue, block 1
// for the largest (kBisectThreads Sturm counts per round, one wave per
// SIMD), block 2 counts the eigenvalues below 0.  A Sturm count is a serial
// recurrence over the n entries; up to kBisectLds entries are first copied
// to LDS, so each step waits on an LDS load rather than a global one.
constexpr int kBisectThreads = 256;
constexpr int64_t kBisectLds = 3072;  // 48 KB of LDS for d and e
__global__ __launch_bounds__(kBisectThreads) void k_bisect(const double* __restrict__ d_g,
                                                           const double* __restrict__ e_g, int64_t n,
                                                           const CheckFlags* fl, double* __restrict__ out) {
    __shared__ double lo_s, hi_s, piv_s;
    __shared__ int cnt[kBisectThreads];
    __shared__ double d_l[kBisectLds], e_l[kBisectLds];
    if (fl->nan_seen) {
        if (threadIdx.x == 0) out[blockIdx.x] = blockIdx.x == 2 ? -1.0 : __builtin_nan("");
        return;
    }
    const bool staged = n <= kBisectLds;
    if (staged)
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            d_l[i] = d_g[i];
            e_l[i] = e_g[i];
        }
    __syncthreads();
    const double* d = staged ? d_l : d_g;
    const double* e = staged ? e_l : e_g;
    double glo = 0, ghi = 0, emax2 = 0;
    if (threadIdx.x == 0) {
        glo = DBL_MAX;
        ghi = -DBL_MAX;
        for (int64_t i = 0; i < n; i++) {
            const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
            glo = fmin(glo, d[i] - r);
            ghi = fmax(ghi, d[i] + r);
            if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
        }
        const double span = fmax(fabs(glo), fabs(ghi));
        glo -= 2.0 * DBL_EPSILON * span * n + DBL_MIN;
        ghi += 2.0 * DBL_EPSILON * span * n + DBL_MIN;
        lo_s = glo;
        hi_s = ghi;
        piv_s = DBL_MIN * fmax(1.0, emax2);
    }
    __syncthreads();
    const double pivmin = piv_s;
    if (blockIdx.x == 2) {
        if (threadIdx.x == 0) out[2] = double(sturm_count(d, e, n, 0.0, pivmin));
        return;
    }
    {
        // block 0: smallest x with count(x) >= 1; block 1: smallest x with count(x) >= n
        const int which = int(blockIdx.x);
        double lo = lo_s, hi = hi_s;
        const int target = which == 0 ? 1 : int(n);
        for (int it = 0; it < 12; it++) {
            const double x = lo + (hi - lo) * double(threadIdx.x + 1) / double(blockDim.x + 1);
            cnt[threadIdx.x] = sturm_count(d, e, n, x, pivmin);
            __syncthreads();
            // bracket: largest point with count < target, smallest with count >= target
            double nlo = lo, nhi = hi;
            for (int q = 0; q < int(blockDim.x); q++) {
                const double xq = lo + (hi - lo) * double(q + 1) / double(blockDim.x + 1);
                if (cnt[q] < target) nlo = xq;
                else {
                    nhi = xq;
                    break;
                }
            }
            __syncthreads();
            lo = nlo;
            hi = nhi;
            if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) break;
        }
        if (threadIdx.x == 0) out[which] = 0.5 * (lo + hi);
    }
}

static int nblocks(int64_t n, int threads, int cap = 4096) {
    return int(std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, cap)));
}

// Check one diagonal block [off, off+n) of C.  Writes chol_ok, n_neg, min, max.
static lc_status check_block(const double* C, int64_t P, int64_t off, int64_t n, hipStream_t s,
                             int32_t* chol_ok, int32_t* n_neg, double* mn, double* mx) {
    if (n == 0) {  // an empty block: nothing to factor, no eigenvalues
        *chol_ok = 1;
        *n_neg = 0;
        *mn = *mx = NAN;
        return LC_OK;
    }
    DevBuf<double> Wb, auxb;
    DevBuf<CheckFlags> flb;
    LC_TRY(Wb.alloc(size_t(n * n), s));
    const int64_t naux = 8 * n + 32;
    LC_TRY(auxb.alloc(size_t(naux), s));
    LC_TRY(flb.alloc(2, s));
    double* W = Wb.get();
    double* aux = auxb.get();
    CheckFlags* fl = flb.get();
    k_zero_flags<<<1, 64, 0, s>>>(fl, 2);
    // two sets of Householder buffers: the launch for column k reads step
    // k-1's set while it fills its own
    double* const v[2] = {aux, aux + n};
    double* const pv[2] = {aux + 2 * n, aux + 3 * n};
    double* d = aux + 4 * n;
    double* e = aux + 5 * n;
    double* const vpp[2] = {aux + 6 * n, aux + 7 * n};  // partial sums of v.p, (n + 3)/4 each
    double* tau = aux + 8 * n;                           // [2]
    double* res = aux + 8 * n + 4;
    // Cholesky
    k_copy_block<<<nblocks(n * n, 256), 256, 0, s>>>(C, P, off, n, W, fl);
    for (int64_t k0 = 0; k0 < n; k0 += kNB) {
        const int nb = int(std::min<int64_t>(kNB, n - k0));
        k_potrf_diag<<<1, 64, 0, s>>>(W, n, k0, nb, fl);
        const int64_t rest = n - k0 - nb;
        if (rest > 0) {
            k_potrf_panel<<<nblocks(rest, 64, 1 << 20), 64, 0, s>>>(W, n, k0, nb, fl);
            const int64_t T = (rest + 63) / 64;
            k_potrf_update<<<int(T * (T + 1) / 2), 256, 0, s>>>(W, n, k0, nb, fl);
        }
    }
    // eigenvalues: fresh copy, tridiagonalise, bisect
    k_copy_block<<<nblocks(n * n, 256), 256, 0, s>>>(C, P, off, n, W, fl + 1);
    HhPending q{nullptr, nullptr, nullptr, nullptr, 0};
    for (int64_t k = 0; k + 2 < n; k++) {
        const int64_t m = n - k - 1;
        const int64_t n1 = (m + kHhRows - 1) / kHhRows;
        const int c = int(k & 1);
        if (m >= 256)
            k_hh_column<4><<<unsigned(n1), 64 * kHhRows * 4, 0, s>>>(W, n, k, q, v[c], tau + c, d, e, pv[c], vpp[c]);
        else
            k_hh_column<1><<<unsigned(n1), 64 * kHhRows, 0, s>>>(W, n, k, q, v[c], tau + c, d, e, pv[c], vpp[c]);
        q = HhPending{v[c], pv[c], tau + c, vpp[c], n1};
    }
    k_hh_tail<<<1, 256, 0, s>>>(W, n, q, d, e);
    k_bisect<<<3, kBisectThreads, 0, s>>>(d, e, n, fl + 1, res);
    CheckFlags hf[2];
    double hr[3];
    LC_TRY_HIP(hipMemcpyAsync(hf, fl, sizeof hf, hipMemcpyDeviceToHost, s));
    LC_TRY_HIP(hipMemcpyAsync(hr, res, sizeof hr, hipMemcpyDeviceToHost, s));
    LC_TRY_HIP(hipStreamSynchronize(s));
    *chol_ok = (!hf[0].nan_seen && !hf[0].chol_fail) ? 1 : 0;
    *n_neg = int32_t(hr[2]);
    *mn = hr[0];
    *mx = hr[1];
    return LC_OK;
}

// The sample covariances of the three estimates, the construction and the
// check; blocks [0, split) and [split, P) of C are checked separately.
static lc_status covariance_impl(const double* xi, int32_t n_mock, int64_t P, int64_t split, double m_a, double m_b,
                                 double M, int32_t precision, double* A, double* B, double* C, lc_cov_report* rep,
                                 hipStream_t s) {
    if (!(M > 0.0)) return fail(LC_ERR_INVALID, "M must be > 0 (or INFINITY)");
    const bool acc32 = (precision & LC_ACC32) != 0;
    precision &= ~LC_ACC32;
    if (precision != LC_FP64 && precision != LC_FP32_MFMA && precision != LC_FP32_MFMA_CHECKED)
        return fail(LC_ERR_INVALID, "precision = %d is not LC_FP64 / LC_FP32_MFMA / LC_FP32_MFMA_CHECKED",
                    precision);
    if (acc32 && precision == LC_FP64) return fail(LC_ERR_INVALID, "LC_ACC32 needs a float32 MFMA precision");
    const int64_t kc = acc32 ? INT64_MAX : int64_t(kKC);
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    (void)ctx;
    const int64_t N = n_mock;
    const int64_t PP = P * P;
    const int64_t W3 = 3 * P;
    const double denom = double(N - 1);
    const int m_inf = std::isinf(M) ? 1 : 0;
    DevBuf<double> meanb, partb, covb, Ab, Bb;
    LC_TRY(meanb.alloc(size_t(W3), s));
    const int64_t nchunk = (N + kMeanRows - 1) / kMeanRows;
    LC_TRY(partb.alloc(size_t(W3 * nchunk), s));
    LC_TRY(covb.alloc(size_t(3 * PP), s));
    if (!A) LC_TRY(Ab.alloc(size_t(PP), s));
    if (!B) LC_TRY(Bb.alloc(size_t(PP), s));
    double* mean = meanb.get();
    double* part = partb.get();
    double* cov = covb.get();
    double* Aw = A ? A : Ab.get();
    double* Bw = B ? B : Bb.get();
    {
        dim3 g(unsigned((W3 + 255) / 256), unsigned(nchunk));
        k_mean_partial<<<g, 256, 0, s>>>(xi, N, W3, part);
        k_mean_final<<<unsigned((W3 + 255) / 256), 256, 0, s>>>(part, nchunk, W3, N, mean);
    }
    const int64_t T64 = (P + 63) / 64;
    auto run_fp64 = [&](double* covbuf) -> lc_status {
        DevBuf<double> dev;
        LC_TRY(dev.alloc(size_t(3 * N * P), s));
        k_dev64<<<nblocks(3 * N * P, 256, 65536), 256, 0, s>>>(xi, mean, N, P, 3, dev.get());
        k_syrk64<<<dim3(unsigned(T64 * (T64 + 1) / 2), 3), 256, 0, s>>>(dev.get(), N, P, denom, covbuf);
        return LC_OK;
    };
    auto run_fp32 = [&](double* covbuf) -> lc_status {
        const int64_t Npad = (N + kKT - 1) / kKT * kKT;
        const int64_t Ppad = (P + kMT - 1) / kMT * kMT;
        DevBuf<float> dev;
        LC_TRY(dev.alloc(size_t(3 * Npad * Ppad), s));
        k_dev32<<<nblocks(3 * Npad * Ppad, 256, 65536), 256, 0, s>>>(xi, mean, N, P, 3, Npad, Ppad, dev.get());
        const int64_t T = Ppad / kMT;
        k_syrk32<<<dim3(unsigned(T * (T + 1) / 2), 3), 256, 0, s>>>(dev.get(), Npad, Ppad, P, kc, denom, covbuf);
        return LC_OK;
    };
    if (precision == LC_FP64) {
        LC_TRY(run_fp64(cov));
    } else {
        LC_TRY(run_fp32(cov));
    }
    k_combine<<<nblocks(PP, 256, 65536), 256, 0, s>>>(cov, PP, m_a, m_b, M, m_inf, Aw, Bw, C);
    double rel[3] = {-1.0, -1.0, -1.0};
    if (precision == LC_FP32_MFMA_CHECKED) {
        DevBuf<double> A64, B64, C64, fpart;
        LC_TRY(A64.alloc(size_t(PP), s));
        LC_TRY(B64.alloc(size_t(PP), s));
        LC_TRY(C64.alloc(size_t(PP), s));
        const int nfb = 512;
        LC_TRY(fpart.alloc(size_t(2 * nfb * 3), s));
        LC_TRY(run_fp64(cov));
        k_combine<<<nblocks(PP, 256, 65536), 256, 0, s>>>(cov, PP, m_a, m_b, M, m_inf, A64.get(), B64.get(),
                                                          C64.get());
        k_frob<<<nfb, 256, 0, s>>>(C, C64.get(), PP, fpart.get());
        k_frob<<<nfb, 256, 0, s>>>(Aw, A64.get(), PP, fpart.get() + 2 * nfb);
        k_frob<<<nfb, 256, 0, s>>>(Bw, B64.get(), PP, fpart.get() + 4 * nfb);
        std::vector<double> h(2 * nfb * 3);
        LC_TRY_HIP(hipMemcpyAsync(h.data(), fpart.get(), sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        A64.reset();
        B64.reset();
        C64.reset();
        fpart.reset();
        LC_TRY_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < 3; q++) {
            double num = 0, den = 0;
            for (int bkt = 0; bkt < nfb; bkt++) {
                num += h[q * 2 * nfb + 2 * bkt];
                den += h[q * 2 * nfb + 2 * bkt + 1];
            }
            rel[q] = den > 0 ? std::sqrt(num / den) : (num > 0 ? INFINITY : 0.0);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LC_ERR_HIP, "covariance launch failed: %s", hipGetErrorString(e));
    meanb.reset();
    partb.reset();
    covb.reset();
    if (rep) {
        rep->rel_frob_vs_fp64[0] = rel[0];
        rep->rel_frob_vs_fp64[1] = rel[1];
        rep->rel_frob_vs_fp64[2] = rel[2];
        LC_TRY(check_block(C, P, 0, split, s, &rep->chol_ok[0], &rep->n_neg_eig[0], &rep->min_eig[0],
                           &rep->max_eig[0]));
        LC_TRY(check_block(C, P, split, P - split, s, &rep->chol_ok[1], &rep->n_neg_eig[1], &rep->min_eig[1],
                           &rep->max_eig[1]));
    }
    return LC_OK;
}


}  // namespace lc

using namespace lc;

extern "C" lc_status lc_covariance(const double* xi, int32_t n_mock, int32_t n_r, int32_t n_mu, int32_t m_a,
                                   double M, int32_t precision, double* A, double* B, double* C,
                                   lc_cov_report* rep, void* stream) {
    clear_error();
    if (!xi || !C) return fail(LC_ERR_INVALID, "xi and C must not be NULL");
    if (n_mock < 2) return fail(LC_ERR_INVALID, "n_mock = %d, need >= 2", n_mock);
    if (n_r < 1 || n_mu < 1 || n_mu > LC_MAX_NMU || int64_t(n_r) * n_mu > LC_MAX_BINS)
        return fail(LC_ERR_INVALID, "bad n_r = %d / n_mu = %d", n_r, n_mu);
    if (m_a < 1) return fail(LC_ERR_INVALID, "m_a = %d, must be >= 1", m_a);
    const int64_t nb0 = int64_t(n_r) * n_mu;
    return covariance_impl(xi, n_mock, nb0 + 3 * int64_t(n_r), nb0, double(m_a), 2.0 * double(m_a), M, precision, A,
                           B, C, rep, (hipStream_t)stream);
}

extern "C" lc_status lc_covariance_general(const double* xi, int32_t n_mock, int32_t P, int32_t n_split, double m_a,
                                           double m_b, double M, int32_t precision, double* A, double* B, double* C,
                                           lc_cov_report* rep, void* stream) {
    clear_error();
    if (!xi || !C) return fail(LC_ERR_INVALID, "xi and C must not be NULL");
    if (n_mock < 2) return fail(LC_ERR_INVALID, "n_mock = %d, need >= 2", n_mock);
    if (P < 1 || P > 4 * LC_MAX_BINS) return fail(LC_ERR_INVALID, "P = %d out of range", P);
    if (n_split < 0 || n_split > P) return fail(LC_ERR_INVALID, "n_split = %d outside [0, P = %d]", n_split, P);
    if (!(m_a > 0.0) || !(m_b > m_a) || !std::isfinite(m_b))
        return fail(LC_ERR_INVALID, "need 0 < m_a < m_b < infinity (got %g, %g)", m_a, m_b);
    return covariance_impl(xi, n_mock, P, n_split, m_a, m_b, M, precision, A, B, C, rep, (hipStream_t)stream);
}

extern "C" lc_status lc_sample_covariance(const double* x, int32_t n_mock, int32_t P, int32_t precision, double* C,
                                          void* stream) {
    clear_error();
    if (!x || !C) return fail(LC_ERR_INVALID, "x and C must not be NULL");
    if (n_mock < 2) return fail(LC_ERR_INVALID, "n_mock = %d, need >= 2", n_mock);
    if (P < 1 || P > 4 * LC_MAX_BINS) return fail(LC_ERR_INVALID, "P = %d out of range", P);
    const bool acc32 = (precision & LC_ACC32) != 0;
    precision &= ~LC_ACC32;
    if (precision != LC_FP64 && precision != LC_FP32_MFMA)
        return fail(LC_ERR_INVALID, "precision = %d is not LC_FP64 / LC_FP32_MFMA", precision);
    if (acc32 && precision == LC_FP64) return fail(LC_ERR_INVALID, "LC_ACC32 needs LC_FP32_MFMA");
    const int64_t kc = acc32 ? INT64_MAX : int64_t(kKC);
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    (void)ctx;
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = n_mock, PL = P;
    const double denom = double(N - 1);
    DevBuf<double> meanb, partb;
    LC_TRY(meanb.alloc(size_t(PL), s));
    const int64_t nchunk = (N + kMeanRows - 1) / kMeanRows;
    LC_TRY(partb.alloc(size_t(PL * nchunk), s));
    double* mean = meanb.get();
    double* part = partb.get();
    {
        dim3 g(unsigned((PL + 255) / 256), unsigned(nchunk));
        k_mean_partial<<<g, 256, 0, s>>>(x, N, PL, part);
        k_mean_final<<<unsigned((PL + 255) / 256), 256, 0, s>>>(part, nchunk, PL, N, mean);
    }
    if (precision == LC_FP64) {
        DevBuf<double> dev;
        LC_TRY(dev.alloc(size_t(N * PL), s));
        k_dev64<<<nblocks(N * PL, 256, 65536), 256, 0, s>>>(x, mean, N, PL, 1, dev.get());
        const int64_t T64 = (PL + 63) / 64;
        k_syrk64<<<dim3(unsigned(T64 * (T64 + 1) / 2), 1), 256, 0, s>>>(dev.get(), N, PL, denom, C);
    } else {
        const int64_t Npad = (N + kKT - 1) / kKT * kKT;
        const int64_t Ppad = (PL + kMT - 1) / kMT * kMT;
        DevBuf<float> dev;
        LC_TRY(dev.alloc(size_t(Npad * Ppad), s));
        k_dev32<<<nblocks(Npad * Ppad, 256, 65536), 256, 0, s>>>(x, mean, N, PL, 1, Npad, Ppad, dev.get());
        const int64_t T = Ppad / kMT;
        k_syrk32<<<dim3(unsigned(T * (T + 1) / 2), 1), 256, 0, s>>>(dev.get(), Npad, Ppad, PL, kc, denom, C);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LC_ERR_HIP, "covariance launch failed: %s", hipGetErrorString(e));
    return LC_OK;
}
