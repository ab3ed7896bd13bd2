// Covariance of the covariance estimates (Sect. 3.2, 3.3) and the summary
// statistics of Sect. 5.3 (chi^2_2, pair-count cost, inverse figure of merit).
//
// For Gaussian data vectors, element (i, j) of a covariance estimated from N
// realisations has variance
//   sample covariance at ratio M:  (C_ii C_jj + C_ij^2) / (N - 1),  C = A + B/M,
//   LC covariance at ratio M:      (D_ii D_jj + D_ij^2 + f^2 (B_ii B_jj + B_ij^2)) / (N - 1),
// with D = A + B/(2 M_a) and f = 1/(2 M_a) - 1/M.  chi^2_2 averages the N = 2
// variances over all elements, each normalised by C^ref_ii C^ref_jj.
#include <cmath>
#include <vector>

#include "lc_internal.hpp"

namespace lc {

__global__ void k_covcov(const double* __restrict__ A, const double* __restrict__ B,
                         const double* __restrict__ Cref, int64_t P, double inv_2ma, double inv_m, double f2,
                         double inv_n1, double* __restrict__ sd_lc, double* __restrict__ sd_smp,
                         double* __restrict__ part) {
    __shared__ double s_lc[256], s_smp[256];
    double acc_lc = 0.0, acc_smp = 0.0;
    const int64_t PP = P * P;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < PP;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = t / P, j = t % P;
        const double aij = A[t], bij = B[t];
        const double aii = A[i * P + i], ajj = A[j * P + j];
        const double bii = B[i * P + i], bjj = B[j * P + j];
        const double dij = aij + bij * inv_2ma, dii = aii + bii * inv_2ma, djj = ajj + bjj * inv_2ma;
        const double cij = aij + bij * inv_m, cii = aii + bii * inv_m, cjj = ajj + bjj * inv_m;
        const double v_lc = dii * djj + dij * dij + f2 * (bii * bjj + bij * bij);
        const double v_smp = cii * cjj + cij * cij;
        const double rii = Cref ? Cref[i * P + i] : cii, rjj = Cref ? Cref[j * P + j] : cjj;
        const double w = 1.0 / (rii * rjj);
        acc_lc += v_lc * w;
        acc_smp += v_smp * w;
        if (sd_lc) sd_lc[t] = sqrt(v_lc * inv_n1);
        if (sd_smp) sd_smp[t] = sqrt(v_smp * inv_n1);
    }
    s_lc[threadIdx.x] = acc_lc;
    s_smp[threadIdx.x] = acc_smp;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s_lc[threadIdx.x] += s_lc[threadIdx.x + o];
            s_smp[threadIdx.x] += s_smp[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s_lc[0];
        part[2 * blockIdx.x + 1] = s_smp[0];
    }
}

}  // namespace lc

using namespace lc;

extern "C" lc_status lc_covcov(const double* A, const double* B, int32_t P, int32_t m_a, double M,
                               const double* Cref, int32_t n_mock, double* sd_lc, double* sd_smp,
                               lc_covcov_report* rep, void* stream) {
    clear_error();
    if (!A || !B) return fail(LC_ERR_INVALID, "A and B must not be NULL");
    if (P < 1 || P > 4 * LC_MAX_BINS) return fail(LC_ERR_INVALID, "P = %d out of range", P);
    if (m_a < 1) return fail(LC_ERR_INVALID, "m_a = %d, must be >= 1", m_a);
    if (!(M > 0.0)) return fail(LC_ERR_INVALID, "M must be > 0 (or INFINITY)");
    if ((sd_lc || sd_smp) && n_mock < 2) return fail(LC_ERR_INVALID, "n_mock = %d, need >= 2", n_mock);
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    (void)ctx;
    hipStream_t s = (hipStream_t)stream;
    const int nblk = 512;
    DevBuf<double> partb;
    LC_TRY(partb.alloc(size_t(2 * nblk), s));
    double* part = partb.get();
    const double inv_m = std::isinf(M) ? 0.0 : 1.0 / M;
    const double f = 1.0 / (2.0 * m_a) - inv_m;
    const double inv_n1 = n_mock >= 2 ? 1.0 / double(n_mock - 1) : 0.0;
    k_covcov<<<nblk, 256, 0, s>>>(A, B, Cref, P, 1.0 / (2.0 * m_a), inv_m, f * f, inv_n1, sd_lc, sd_smp, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LC_ERR_HIP, "covcov launch failed: %s", hipGetErrorString(e));
    if (rep) {
        std::vector<double> h(2 * nblk);
        LC_TRY_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        LC_TRY_HIP(hipStreamSynchronize(s));
        double lc_sum = 0.0, smp_sum = 0.0;
        for (int b = 0; b < nblk; b++) {
            lc_sum += h[2 * b];
            smp_sum += h[2 * b + 1];
        }
        const double n2 = double(P) * double(P);
        rep->chi2_2_lc = lc_sum / n2;
        rep->chi2_2_smp = smp_sum / n2;
        // Sect. 2.3: two split estimates with ratio M_a, DD counted once:
        // DD (1) + 2 x (DR 2 M_a + split RR M_a) in units of N_d^2 / 2
        rep->cost_lc = 1.0 + 6.0 * double(m_a);
        rep->cost_smp = std::isinf(M) ? INFINITY : 1.0 + 3.0 * M;
        rep->ifom_lc = rep->cost_lc * rep->chi2_2_lc;
        rep->ifom_smp = rep->cost_smp * rep->chi2_2_smp;
        rep->gain = rep->ifom_smp / rep->ifom_lc;
    }
    return LC_OK;
}
