// Co-added pair counts and linear maps of data vectors and covariances.
//
// Co-adding the counts of adjacent bins gives wider r bins and, summed over
// all mu bins, the one-dimensional correlation function (Sect. 4.3); the
// co-added counts go through the estimator like the original ones.  A linear
// map y = T x in which every input element feeds at most one output (with a
// weight) re-bins or selects the elements of a data vector; the covariance
// of the mapped vector is T C T^T.  The linear construction is linear in the
// covariances, so A, B and C^LC can be mapped after they are built (Sect. 2.3;
// Sect. 5.3 re-bins the covariance matrices this way).
//
// Counts are summed in uint64 (exact).  Maps sum in float64 in increasing
// input order, each output as sum over its members a of w_a x_a (vectors) or
// sum_a w_a (sum_b w_b X_ab) (matrices).
#include <algorithm>
#include <cmath>
#include <vector>

#include "lc_internal.hpp"

namespace lc {

namespace {

// out[t][k2][m2] = sum of in[t][k][m] over k in group k2 (w_r wide, the last
// one ragged) and m in group m2 (w_mu wide).  One thread per output bin.
__global__ void k_rebin_counts(const unsigned long long* __restrict__ in, int64_t n_out, int32_t n_r, int32_t n_mu,
                               int32_t w_r, int32_t w_mu, int32_t n_r2, int32_t n_mu2,
                               unsigned long long* __restrict__ out) {
    for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < n_out;
         o += int64_t(gridDim.x) * blockDim.x) {
        const int32_t m2 = int32_t(o % n_mu2);
        const int64_t r = o / n_mu2;
        const int32_t k2 = int32_t(r % n_r2);
        const int64_t t = r / n_r2;
        const int32_t k0 = k2 * w_r;
        const int32_t k1 = min(k0 + w_r, n_r);
        const unsigned long long* src = in + t * int64_t(n_r) * n_mu;
        unsigned long long s = 0;
        for (int32_t k = k0; k < k1; k++)
            for (int32_t m = m2 * w_mu; m < (m2 + 1) * w_mu; m++) s += src[int64_t(k) * n_mu + m];
        out[o] = s;
    }
}

// y[n][g] = sum over members a of group g (increasing) of w_a x[n][a].
__global__ void k_map_vectors(const double* __restrict__ x, int64_t n_vec, int64_t ld_x, int32_t P_out,
                              const int32_t* __restrict__ goff, const int32_t* __restrict__ gmem,
                              const double* __restrict__ gw, int64_t ld_y, double* __restrict__ y) {
#pragma clang fp contract(off)
    const int64_t tot = n_vec * P_out;
    for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < tot;
         o += int64_t(gridDim.x) * blockDim.x) {
        const int32_t g = int32_t(o % P_out);
        const int64_t n = o / P_out;
        const double* xr = x + n * ld_x;
        double s = 0.0;
        for (int32_t q = goff[g]; q < goff[g + 1]; q++) s = s + gw[q] * xr[gmem[q]];
        y[n * ld_y + g] = s;
    }
}

// Y[g][h] = sum_a w_a (sum_b w_b X[a][b]), a over group g and b over group h
// in increasing order.  One thread per output element; every input element
// is read by exactly one thread, so the launch streams X once.
__global__ void k_map_matrix(const double* __restrict__ X, int32_t P_in, int32_t P_out,
                             const int32_t* __restrict__ goff, const int32_t* __restrict__ gmem,
                             const double* __restrict__ gw, double* __restrict__ Y) {
#pragma clang fp contract(off)
    const int64_t tot = int64_t(P_out) * P_out;
    for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < tot;
         o += int64_t(gridDim.x) * blockDim.x) {
        const int32_t h = int32_t(o % P_out);
        const int32_t g = int32_t(o / P_out);
        double s = 0.0;
        for (int32_t qa = goff[g]; qa < goff[g + 1]; qa++) {
            const double* row = X + int64_t(gmem[qa]) * P_in;
            double r = 0.0;
            for (int32_t qb = goff[h]; qb < goff[h + 1]; qb++) r = r + gw[qb] * row[gmem[qb]];
            s = s + gw[qa] * r;
        }
        Y[o] = s;
    }
}

int grid_for(int64_t n, int threads) {
    return int(std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, 65536)));
}

// Host CSR of a map: outputs in order, members of each in increasing input
// order.  Validates group ids and weights.
lc_status build_map(const int32_t* group, const double* weight, int32_t P_in, int32_t P_out,
                    std::vector<int32_t>& goff, std::vector<int32_t>& gmem, std::vector<double>& gw) {
    if (!group || !weight) return fail(LC_ERR_INVALID, "group and weight must not be NULL");
    goff.assign(size_t(P_out) + 1, 0);
    for (int32_t i = 0; i < P_in; i++) {
        const int32_t g = group[i];
        if (g < -1 || g >= P_out) return fail(LC_ERR_INVALID, "group[%d] = %d outside [-1, %d)", i, g, P_out);
        if (g >= 0) {
            if (!std::isfinite(weight[i])) return fail(LC_ERR_INVALID, "weight[%d] is not finite", i);
            goff[size_t(g) + 1]++;
        }
    }
    for (int32_t g = 0; g < P_out; g++) goff[size_t(g) + 1] += goff[g];
    gmem.assign(size_t(goff[P_out]), 0);
    gw.assign(size_t(goff[P_out]), 0.0);
    std::vector<int32_t> fill(goff.begin(), goff.end() - 1);
    for (int32_t i = 0; i < P_in; i++) {
        const int32_t g = group[i];
        if (g < 0) continue;
        gmem[size_t(fill[g])] = i;
        gw[size_t(fill[g])] = weight[i];
        fill[g]++;
    }
    return LC_OK;
}

// Stage the CSR to the device; one allocation, freed by the caller.
lc_status stage_map(DeviceCtx* ctx, hipStream_t s, const std::vector<int32_t>& goff, std::vector<int32_t>& gmem,
                    std::vector<double>& gw, void** dev, const int32_t** d_off, const int32_t** d_mem,
                    const double** d_w) {
    if (gmem.empty()) {  // a map that drops everything: one unused entry keeps the arrays non-empty
        gmem.push_back(0);
        gw.push_back(0.0);
    }
    Stager stg(ctx);
    const size_t o_off = stg.push(goff.data(), sizeof(int32_t) * goff.size());
    const size_t o_mem = stg.push(gmem.data(), sizeof(int32_t) * gmem.size());
    const size_t o_w = stg.push(gw.data(), sizeof(double) * gw.size());
    LC_TRY(stg.commit(s, dev));
    auto* base = static_cast<unsigned char*>(*dev);
    *d_off = reinterpret_cast<const int32_t*>(base + o_off);
    *d_mem = reinterpret_cast<const int32_t*>(base + o_mem);
    *d_w = reinterpret_cast<const double*>(base + o_w);
    return LC_OK;
}

}  // namespace

}  // namespace lc

using namespace lc;

extern "C" lc_status lc_rebin_counts(const uint64_t* counts, int32_t n_tasks, int32_t n_r, int32_t n_mu, int32_t w_r,
                                     int32_t w_mu, uint64_t* out, void* stream) {
    clear_error();
    if (n_tasks < 0) return fail(LC_ERR_INVALID, "n_tasks = %d < 0", n_tasks);
    if (n_r < 1 || n_mu < 1 || int64_t(n_r) * n_mu > LC_MAX_BINS)
        return fail(LC_ERR_INVALID, "bad n_r = %d / n_mu = %d", n_r, n_mu);
    if (w_r < 1 || w_r > n_r) return fail(LC_ERR_INVALID, "w_r = %d outside [1, n_r = %d]", w_r, n_r);
    if (w_mu < 1 || n_mu % w_mu != 0)
        return fail(LC_ERR_INVALID, "w_mu = %d must be >= 1 and divide n_mu = %d", w_mu, n_mu);
    if (n_tasks == 0) return LC_OK;
    if (!counts || !out) return fail(LC_ERR_INVALID, "counts and out must not be NULL");
    if (static_cast<const void*>(counts) == static_cast<const void*>(out))
        return fail(LC_ERR_INVALID, "out must not alias counts");
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    (void)ctx;
    hipStream_t s = (hipStream_t)stream;
    const int32_t n_r2 = (n_r + w_r - 1) / w_r, n_mu2 = n_mu / w_mu;
    const int64_t n_out = int64_t(n_tasks) * n_r2 * n_mu2;
    k_rebin_counts<<<grid_for(n_out, 256), 256, 0, s>>>(reinterpret_cast<const unsigned long long*>(counts), n_out,
                                                        n_r, n_mu, w_r, w_mu, n_r2, n_mu2,
                                                        reinterpret_cast<unsigned long long*>(out));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LC_ERR_HIP, "rebin launch failed: %s", hipGetErrorString(e));
    return LC_OK;
}

extern "C" lc_status lc_map_vectors(const double* x, int64_t n_vec, int32_t P_in, int64_t ld_x, const int32_t* group,
                                    const double* weight, int32_t P_out, double* y, int64_t ld_y, void* stream) {
    clear_error();
    if (n_vec < 0) return fail(LC_ERR_INVALID, "n_vec < 0");
    if (P_in < 1 || P_out < 1) return fail(LC_ERR_INVALID, "P_in = %d and P_out = %d must be >= 1", P_in, P_out);
    if (ld_x == 0) ld_x = P_in;
    if (ld_y == 0) ld_y = P_out;
    if (ld_x < P_in || ld_y < P_out) return fail(LC_ERR_INVALID, "ld_x < P_in or ld_y < P_out");
    std::vector<int32_t> goff, gmem;
    std::vector<double> gw;
    LC_TRY(build_map(group, weight, P_in, P_out, goff, gmem, gw));
    if (n_vec == 0) return LC_OK;
    if (!x || !y) return fail(LC_ERR_INVALID, "x and y must not be NULL");
    if (static_cast<const void*>(x) == static_cast<const void*>(y))
        return fail(LC_ERR_INVALID, "y must not alias x");
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    hipStream_t s = (hipStream_t)stream;
    void* dev = nullptr;
    const int32_t *d_off, *d_mem;
    const double* d_w;
    LC_TRY(stage_map(ctx, s, goff, gmem, gw, &dev, &d_off, &d_mem, &d_w));
    k_map_vectors<<<grid_for(n_vec * P_out, 256), 256, 0, s>>>(x, n_vec, ld_x, P_out, d_off, d_mem, d_w, ld_y, y);
    hipError_t e = hipGetLastError();
    dev_free(dev, s);
    if (e != hipSuccess) return fail(LC_ERR_HIP, "map launch failed: %s", hipGetErrorString(e));
    return LC_OK;
}

extern "C" lc_status lc_map_matrix(const double* X, int32_t P_in, const int32_t* group, const double* weight,
                                   int32_t P_out, double* Y, void* stream) {
    clear_error();
    if (P_in < 1 || P_out < 1) return fail(LC_ERR_INVALID, "P_in = %d and P_out = %d must be >= 1", P_in, P_out);
    std::vector<int32_t> goff, gmem;
    std::vector<double> gw;
    LC_TRY(build_map(group, weight, P_in, P_out, goff, gmem, gw));
    if (!X || !Y) return fail(LC_ERR_INVALID, "X and Y must not be NULL");
    if (static_cast<const void*>(X) == static_cast<const void*>(Y))
        return fail(LC_ERR_INVALID, "Y must not alias X");
    DeviceCtx* ctx;
    LC_TRY(get_ctx(&ctx));
    hipStream_t s = (hipStream_t)stream;
    void* dev = nullptr;
    const int32_t *d_off, *d_mem;
    const double* d_w;
    LC_TRY(stage_map(ctx, s, goff, gmem, gw, &dev, &d_off, &d_mem, &d_w));
    k_map_matrix<<<grid_for(int64_t(P_out) * P_out, 256), 256, 0, s>>>(X, P_in, P_out, d_off, d_mem, d_w, Y);
    hipError_t e = hipGetLastError();
    dev_free(dev, s);
    if (e != hipSuccess) return fail(LC_ERR_HIP, "map launch failed: %s", hipGetErrorString(e));
    return LC_OK;
}

// ---------------------------------------------------------------------------
// maps of the data vector (host): the inputs of lc_map_vectors / lc_map_matrix
// ---------------------------------------------------------------------------

extern "C" lc_status lc_map_multipoles(int32_t n_r, int32_t n_mu, int32_t w, int32_t r_lo, int32_t r_hi,
                                       int32_t ell_mask, int32_t* group, double* weight, int32_t* P_out) {
    clear_error();
    if (!group || !weight || !P_out) return fail(LC_ERR_INVALID, "group, weight and P_out must not be NULL");
    if (n_r < 1 || n_mu < 1 || int64_t(n_r) * n_mu > LC_MAX_BINS)
        return fail(LC_ERR_INVALID, "bad n_r = %d / n_mu = %d", n_r, n_mu);
    if (!(0 <= r_lo && r_lo < r_hi && r_hi <= n_r) || w < 1)
        return fail(LC_ERR_INVALID, "bad r range [%d, %d) or width %d", r_lo, r_hi, w);
    if (ell_mask < 1 || ell_mask > 7) return fail(LC_ERR_INVALID, "ell_mask = %d, must select l = 0, 2 or 4", ell_mask);
    const int32_t P = n_r * n_mu + 3 * n_r;
    for (int32_t i = 0; i < P; i++) {
        group[i] = -1;
        weight[i] = 0.0;
    }
    // the output mean of a group of w adjacent r bins (the last group of a
    // range that w does not divide is narrower)
    const int32_t n_out = (r_hi - r_lo + w - 1) / w;
    int32_t j = 0;
    for (int li = 0; li < 3; li++) {
        if (!(ell_mask & (1 << li))) continue;
        for (int32_t k = r_lo; k < r_hi; k++) {
            const int32_t gk = (k - r_lo) / w;
            const int32_t size = std::min(w, r_hi - r_lo - gk * w);
            const int32_t i = n_r * n_mu + li * n_r + k;
            group[i] = j * n_out + gk;
            weight[i] = 1.0 / double(size);
        }
        j++;
    }
    *P_out = j * n_out;
    return LC_OK;
}

extern "C" lc_status lc_map_projected(int32_t n_rp, int32_t n_pi, double pi_max, int32_t* group, double* weight,
                                      int32_t* P_out) {
    clear_error();
    if (!group || !weight || !P_out) return fail(LC_ERR_INVALID, "group, weight and P_out must not be NULL");
    if (n_rp < 1 || n_pi < 1 || int64_t(n_rp) * n_pi > LC_MAX_BINS)
        return fail(LC_ERR_INVALID, "bad n_rp = %d / n_pi = %d", n_rp, n_pi);
    if (!(pi_max > 0.0) || !std::isfinite(pi_max)) return fail(LC_ERR_INVALID, "pi_max must be finite and > 0");
    const int32_t nb = n_rp * n_pi, P = nb + 3 * n_rp;
    // w_p(r_p) = 2 sum_m xi(r_p, pi_m) dpi with dpi = pi_max / n_pi, xi held
    // constant within a pi bin
    const double coef = 2.0 * pi_max / double(n_pi);
    for (int32_t i = 0; i < P; i++) {
        group[i] = i < nb ? i / n_pi : -1;
        weight[i] = i < nb ? coef : 0.0;
    }
    *P_out = n_rp;
    return LC_OK;
}

extern "C" lc_status lc_map_rebin_blocks(int32_t n_blocks, int32_t n, int32_t w, int32_t* group, double* weight,
                                         int32_t* P_out) {
    clear_error();
    if (!group || !weight || !P_out) return fail(LC_ERR_INVALID, "group, weight and P_out must not be NULL");
    if (w < 1 || n < 1 || n_blocks < 1 || int64_t(n_blocks) * n > int64_t(4) * LC_MAX_BINS)
        return fail(LC_ERR_INVALID, "bad block map sizes (%d blocks of %d, width %d)", n_blocks, n, w);
    const int32_t n_out = (n + w - 1) / w;
    for (int32_t b = 0; b < n_blocks; b++)
        for (int32_t k = 0; k < n; k++) {
            const int32_t gk = k / w;
            group[b * n + k] = b * n_out + gk;
            weight[b * n + k] = 1.0 / double(std::min(w, n - gk * w));
        }
    *P_out = n_blocks * n_out;
    return LC_OK;
}
