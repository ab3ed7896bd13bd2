// Split Landy-Szalay estimates and Legendre multipoles (Sect. 2.1, 2.3, 4.3).
//
// For each mock: dd = DD/(N_d(N_d-1)/2), dr_i = DR_i/(N_d N_r,i),
// rr_i = RR_i/(N_r,i(N_r,i-1)/2), and xi = (dd - (2/M) sum dr_i)/((1/M) sum rr_i) + 1
// for (D,R1) and (D,R2) with M = 1 and for (D, R1 u R2) with M = 2, where the
// M = 2 estimate reuses the two subsets' counts (pairs across subsets are not
// part of the split estimator).  Multipoles: xi_l(r) = sum_m W_lm xi(r, mu_m),
// W_lm = (2l+1) * integral of P_l over mu bin m of [0, 1].
#include <cmath>
#include <vector>

#include "lc_internal.hpp"

namespace lc {

__global__ void k_xi(const unsigned long long* __restrict__ counts, const int32_t* __restrict__ est,
                     const double* __restrict__ norm, const double* __restrict__ W, int32_t n_mock,
                     int32_t n_r, int32_t n_mu, double* __restrict__ xi) {
#pragma clang fp contract(off)
    const int64_t idx = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (idx >= int64_t(n_mock) * n_r) return;
    const int mk = int(idx / n_r), k = int(idx % n_r);
    const int64_t nb = int64_t(n_r) * n_mu;
    const int64_t P = nb + 3 * int64_t(n_r);
    const int32_t* e = est + 5 * int64_t(mk);
    const double* nr = norm + 5 * int64_t(mk);
    const unsigned long long* cDD = counts + e[0] * nb + int64_t(k) * n_mu;
    const unsigned long long* cDR1 = counts + e[1] * nb + int64_t(k) * n_mu;
    const unsigned long long* cDR2 = counts + e[2] * nb + int64_t(k) * n_mu;
    const unsigned long long* cRR1 = counts + e[3] * nb + int64_t(k) * n_mu;
    const unsigned long long* cRR2 = counts + e[4] * nb + int64_t(k) * n_mu;
    double* out = xi + int64_t(mk) * 3 * P;
    double mp[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const double nan = __builtin_nan("");
    for (int m = 0; m < n_mu; m++) {
        const double dd = double(cDD[m]) / nr[0];
        const double dr1 = double(cDR1[m]) / nr[1];
        const double dr2 = double(cDR2[m]) / nr[2];
        const double rr1 = double(cRR1[m]) / nr[3];
        const double rr2 = double(cRR2[m]) / nr[4];
        double x[3];
        {   // M = 1 with R1, then with R2
            const double den1 = 1.0 * rr1, den2 = 1.0 * rr2;
            x[0] = den1 == 0.0 ? nan : (dd - 2.0 * dr1) / den1 + 1.0;
            x[1] = den2 == 0.0 ? nan : (dd - 2.0 * dr2) / den2 + 1.0;
        }
        {   // M = 2, split over R1 and R2
            const double sdr = dr1 + dr2, srr = rr1 + rr2;
            const double den = 0.5 * srr;
            x[2] = den == 0.0 ? nan : (dd - 1.0 * sdr) / den + 1.0;
        }
        for (int q = 0; q < 3; q++) {
            out[q * P + int64_t(k) * n_mu + m] = x[q];
            for (int l = 0; l < 3; l++) mp[q][l] = mp[q][l] + W[l * n_mu + m] * x[q];
        }
    }
    for (int q = 0; q < 3; q++)
        for (int l = 0; l < 3; l++) out[q * P + nb + int64_t(l) * n_r + k] = mp[q][l];
}

// One split estimate per mock with M random sub-catalogues (the sample
// covariance's estimator, Sect. 2.1-2.2): est row = [DD, DR_1..DR_M,
// RR_1..RR_M], norm row alike.  xi = (dd - (2/M) sum dr_i) / ((1/M) sum rr_i) + 1,
// the sums taken in subset order.  Output row n at xi + n ld (xi(r, mu) then
// the multipoles, P values).
__global__ void k_xi_split(const unsigned long long* __restrict__ counts, const int32_t* __restrict__ est,
                           const double* __restrict__ norm, const double* __restrict__ W, int32_t n_mock,
                           int32_t n_sub, int32_t n_r, int32_t n_mu, int64_t ld, double* __restrict__ xi) {
#pragma clang fp contract(off)
    const int64_t idx = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (idx >= int64_t(n_mock) * n_r) return;
    const int mk = int(idx / n_r), k = int(idx % n_r);
    const int64_t nb = int64_t(n_r) * n_mu;
    const int64_t P = nb + 3 * int64_t(n_r);
    const int64_t w = 1 + 2 * int64_t(n_sub);
    const int32_t* e = est + w * mk;
    const double* nr = norm + w * mk;
    const double two_over_m = 2.0 / double(n_sub), one_over_m = 1.0 / double(n_sub);
    double* out = xi + int64_t(mk) * ld;
    double mp[3] = {0, 0, 0};
    const double nan = __builtin_nan("");
    for (int m = 0; m < n_mu; m++) {
        const int64_t off = int64_t(k) * n_mu + m;
        const double dd = double(counts[e[0] * nb + off]) / nr[0];
        double sdr = 0.0, srr = 0.0;
        for (int i = 0; i < n_sub; i++) {
            sdr = sdr + double(counts[e[1 + i] * nb + off]) / nr[1 + i];
            srr = srr + double(counts[e[1 + n_sub + i] * nb + off]) / nr[1 + n_sub + i];
        }
        const double den = one_over_m * srr;
        const double x = den == 0.0 ? nan : (dd - two_over_m * sdr) / den + 1.0;
        out[off] = x;
        for (int l = 0; l < 3; l++) mp[l] = mp[l] + W[l * n_mu + m] * x;
    }
    for (int l = 0; l < 3; l++) out[nb + int64_t(l) * n_r + k] = mp[l];
}

// Integral of P_l from 0 to x, l = 0, 2, 4 (P_2 = (3x^2-1)/2, P_4 = (35x^4-30x^2+3)/8).
static double legendre_integral(int l, double x) {
    const double x2 = x * x;
    switch (l) {
        case 0: return x;
        case 2: return 0.5 * x * (x2 - 1.0);
        default: return x * (x2 * (7.0 * x2 - 10.0) + 3.0) / 8.0;
    }
}

static std::vector<double> legendre_weights(int n_mu) {
    std::vector<double> W(3 * size_t(n_mu));
    for (int li = 0; li < 3; li++) {
        const int l = 2 * li;
        for (int m = 0; m < n_mu; m++) {
            const double a = double(m) / n_mu, b = double(m + 1) / n_mu;
            W[li * size_t(n_mu) + m] = (2 * l + 1) * (legendre_integral(l, b) - legendre_integral(l, a));
        }
    }
    return W;
}

}  // namespace lc

using namespace lc;

extern "C" lc_status lc_xi_multipoles(const uint64_t* counts, const lc_task* tasks, int32_t n_tasks,
                                      const int64_t* cat_sizes, int32_t n_cat, const int32_t* est,
                                      int32_t n_mock, int32_t n_r, int32_t n_mu, double* xi, void* stream) {
    clear_error();
    if (n_mock < 0) return fail(LC_ERR_INVALID, "n_mock < 0");
    if (n_mock == 0) return LC_OK;
    if (!counts || !tasks || !cat_sizes || !est || !xi) return fail(LC_ERR_INVALID, "NULL argument");
    if (n_r < 1 || n_mu < 1 || n_mu > LC_MAX_NMU || int64_t(n_r) * n_mu > LC_MAX_BINS)
        return fail(LC_ERR_INVALID, "bad n_r = %d / n_mu = %d", n_r, n_mu);
    if (n_tasks < 1 || n_cat < 1) return fail(LC_ERR_INVALID, "n_tasks and n_cat must be >= 1");
    std::vector<double> norm(5 * size_t(n_mock));
    for (int32_t m = 0; m < n_mock; m++) {
        const int32_t* e = est + 5 * size_t(m);
        for (int q = 0; q < 5; q++)
            if (e[q] < 0 || e[q] >= n_tasks)
                return fail(LC_ERR_INVALID, "mock %d: task id %d out of range", m, e[q]);
        const lc_task DD = tasks[e[0]], DR1 = tasks[e[1]], DR2 = tasks[e[2]], RR1 = tasks[e[3]],
                      RR2 = tasks[e[4]];
        const int32_t D = DD.cat_a, R1 = DR1.cat_b, R2 = DR2.cat_b;
        if (DD.cat_b != D || DR1.cat_a != D || DR2.cat_a != D || DR1.cat_b == D || DR2.cat_b == D ||
            RR1.cat_a != R1 || RR1.cat_b != R1 || RR2.cat_a != R2 || RR2.cat_b != R2)
            return fail(LC_ERR_INVALID,
                        "mock %d: tasks are not DD=(D,D), DR1=(D,R1), DR2=(D,R2), RR1=(R1,R1), RR2=(R2,R2)", m);
        for (int32_t c : {D, R1, R2})
            if (c < 0 || c >= n_cat) return fail(LC_ERR_INVALID, "mock %d: catalogue %d out of range", m, c);
        const int64_t nd = cat_sizes[D], n1 = cat_sizes[R1], n2 = cat_sizes[R2];
        if (nd < 2 || n1 < 2 || n2 < 2)
            return fail(LC_ERR_INVALID, "mock %d: every catalogue needs >= 2 points", m);
        if (nd >= (int64_t(1) << 26) || n1 >= (int64_t(1) << 26) || n2 >= (int64_t(1) << 26))
            return fail(LC_ERR_OVERFLOW, "mock %d: catalogue too large for exact normalisation", m);
        double* nr = norm.data() + 5 * size_t(m);
        nr[0] = double(nd * (nd - 1)) / 2.0;
        nr[1] = double(nd) * double(n1);
        nr[2] = double(nd) * double(n2);
        nr[3] = double(n1 * (n1 - 1)) / 2.0;
        nr[4] = double(n2 * (n2 - 1)) / 2.0;
    }
    const std::vector<double> W = legendre_weights(n_mu);
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    hipStream_t s = (hipStream_t)stream;
    void* dev = nullptr;
    Stager stg(ctx);
    size_t o_est = stg.push(est, sizeof(int32_t) * 5 * size_t(n_mock));
    size_t o_norm = stg.push(norm.data(), sizeof(double) * norm.size());
    size_t o_w = stg.push(W.data(), sizeof(double) * W.size());
    LC_TRY(stg.commit(s, &dev));
    auto* base = static_cast<unsigned char*>(dev);
    const int64_t n = int64_t(n_mock) * n_r;
    const int threads = 128;
    k_xi<<<int((n + threads - 1) / threads), threads, 0, s>>>(
        reinterpret_cast<const unsigned long long*>(counts), reinterpret_cast<const int32_t*>(base + o_est),
        reinterpret_cast<const double*>(base + o_norm), reinterpret_cast<const double*>(base + o_w), n_mock,
        n_r, n_mu, xi);
    hipError_t e = hipGetLastError();
    dev_free(dev, s);
    if (e != hipSuccess) return fail(LC_ERR_HIP, "xi launch failed: %s", hipGetErrorString(e));
    return LC_OK;
}

extern "C" lc_status lc_xi_split(const uint64_t* counts, const lc_task* tasks, int32_t n_tasks,
                                 const int64_t* cat_sizes, int32_t n_cat, const int32_t* est, int32_t n_sub,
                                 int32_t n_mock, int32_t n_r, int32_t n_mu, double* xi, int64_t ld_xi,
                                 void* stream) {
    clear_error();
    if (n_mock < 0) return fail(LC_ERR_INVALID, "n_mock < 0");
    if (n_mock == 0) return LC_OK;
    if (!counts || !tasks || !cat_sizes || !est || !xi) return fail(LC_ERR_INVALID, "NULL argument");
    const int64_t P = int64_t(n_r) * n_mu + 3 * int64_t(n_r);
    if (ld_xi == 0) ld_xi = P;
    if (ld_xi < P) return fail(LC_ERR_INVALID, "ld_xi = %lld < P = %lld", (long long)ld_xi, (long long)P);
    if (n_sub < 1 || n_sub > 4096) return fail(LC_ERR_INVALID, "n_sub = %d out of [1, 4096]", n_sub);
    if (n_r < 1 || n_mu < 1 || n_mu > LC_MAX_NMU || int64_t(n_r) * n_mu > LC_MAX_BINS)
        return fail(LC_ERR_INVALID, "bad n_r = %d / n_mu = %d", n_r, n_mu);
    if (n_tasks < 1 || n_cat < 1) return fail(LC_ERR_INVALID, "n_tasks and n_cat must be >= 1");
    const size_t w = 1 + 2 * size_t(n_sub);
    std::vector<double> norm(w * size_t(n_mock));
    for (int32_t m = 0; m < n_mock; m++) {
        const int32_t* e = est + w * size_t(m);
        for (size_t q = 0; q < w; q++)
            if (e[q] < 0 || e[q] >= n_tasks) return fail(LC_ERR_INVALID, "mock %d: task id %d out of range", m, e[q]);
        const lc_task DD = tasks[e[0]];
        const int32_t D = DD.cat_a;
        if (DD.cat_b != D || D < 0 || D >= n_cat)
            return fail(LC_ERR_INVALID, "mock %d: the first task is not DD = (D, D)", m);
        const int64_t nd = cat_sizes[D];
        if (nd < 2 || nd >= (int64_t(1) << 26))
            return fail(LC_ERR_INVALID, "mock %d: data catalogue size %lld outside [2, 2^26)", m, (long long)nd);
        double* nr = norm.data() + w * size_t(m);
        nr[0] = double(nd * (nd - 1)) / 2.0;
        for (int32_t i = 0; i < n_sub; i++) {
            const lc_task DR = tasks[e[1 + i]], RR = tasks[e[1 + n_sub + i]];
            const int32_t R = DR.cat_b;
            if (DR.cat_a != D || R == D || R < 0 || R >= n_cat || RR.cat_a != R || RR.cat_b != R)
                return fail(LC_ERR_INVALID, "mock %d subset %d: tasks are not DR = (D, R), RR = (R, R)", m, i);
            const int64_t n1 = cat_sizes[R];
            if (n1 < 2 || n1 >= (int64_t(1) << 26))
                return fail(LC_ERR_INVALID, "mock %d subset %d: size %lld outside [2, 2^26)", m, i, (long long)n1);
            nr[1 + i] = double(nd) * double(n1);
            nr[1 + n_sub + i] = double(n1 * (n1 - 1)) / 2.0;
        }
    }
    const std::vector<double> W = legendre_weights(n_mu);
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    hipStream_t s = (hipStream_t)stream;
    void* dev = nullptr;
    Stager stg(ctx);
    size_t o_est = stg.push(est, sizeof(int32_t) * w * size_t(n_mock));
    size_t o_norm = stg.push(norm.data(), sizeof(double) * norm.size());
    size_t o_w = stg.push(W.data(), sizeof(double) * W.size());
    LC_TRY(stg.commit(s, &dev));
    auto* base = static_cast<unsigned char*>(dev);
    const int64_t n = int64_t(n_mock) * n_r;
    const int threads = 128;
    k_xi_split<<<int((n + threads - 1) / threads), threads, 0, s>>>(
        reinterpret_cast<const unsigned long long*>(counts), reinterpret_cast<const int32_t*>(base + o_est),
        reinterpret_cast<const double*>(base + o_norm), reinterpret_cast<const double*>(base + o_w), n_mock,
        n_sub, n_r, n_mu, ld_xi, xi);
    hipError_t e = hipGetLastError();
    dev_free(dev, s);
    if (e != hipSuccess) return fail(LC_ERR_HIP, "xi launch failed: %s", hipGetErrorString(e));
    return LC_OK;
}
