/*
 * Brute-force (r, mu) pair counter.  TEST INFRASTRUCTURE ONLY: this is the
 * oracle that the GPU path is checked against.  Only tests, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product path
 * never does.  It shares no code with the GPU library.
 *
 * What it computes (Sect. 2.1, the pair counts DD, DR_i and RR_i that feed
 * the split Landy-Szalay estimator, binned in separation r and in mu, the
 * cosine between the line of sight and the pair separation as in Sect. 4.3):
 *
 *   for every unordered pair i<j of one catalogue (auto = 1), or every pair
 *   (i in A, j in B) of two catalogues (auto = 0):
 *     s  = x_j - x_i per axis, in int64; in a periodic box of side L the
 *          minimal image is taken: s >= L/2 -> s - L, s < -L/2 -> s + L
 *     d2 = s.s (exact: |s| < 2^26 so d2 < 2^53)
 *     r-bin k: e_k^2 <= d2 < e_{k+1}^2, pairs outside [e_0, e_n) dropped
 *     mu-bin m, plane-parallel (line of sight = z axis):
 *          the largest m in [0, n_mu-1] with m^2 d2 <= n_mu^2 s_z^2,
 *          i.e. floor(n_mu |s_z| / d) clamped to n_mu - 1; d2 = 0 -> m = 0
 *     mu-bin m, midpoint line of sight (observer at the origin):
 *          l = x_i + x_j (twice the midpoint), p = s.l, q = l.l,
 *          the largest m in [0, n_mu-1] with m^2 d2 q <= n_mu^2 p^2;
 *          d2 = 0 or q = 0 -> m = 0
 *     counts[k][m] += 1
 *
 *   (r_p, pi) binning (plane-parallel along z; the binning of the projected
 *   correlation function, Sect. 2.3): the same loops with
 *     r_p-bin k: e_k^2 <= s_x^2 + s_y^2 < e_{k+1}^2
 *     pi-bin m: pairs with |s_z| >= pi_max dropped, else
 *          m = floor(n_pi |s_z| / pi_max) (integer division)
 *
 * All comparisons are exact integer arithmetic in unsigned 128 bits.  The
 * loops are the plain O(N_a N_b) enumeration, parallelised over i only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

static inline int64_t wrap(int64_t s, int64_t box) {
    if (box > 0) {
        if (s >= box / 2) s -= box;
        else if (s < -(box / 2)) s += box;
    }
    return s;
}

static inline uint64_t uabs64(int64_t v) { return v < 0 ? (uint64_t)(-v) : (uint64_t)v; }

/* r-bin: -1 if not binned */
static inline int r_bin(uint64_t d2, const uint64_t* e2, int n_r) {
    if (d2 < e2[0] || d2 >= e2[n_r]) return -1;
    int k = 0;
    while (d2 >= e2[k + 1]) k++;
    return k;
}

static inline int mu_bin_z(uint64_t d2, int64_t sz, int n_mu) {
    if (d2 == 0) return 0;
    uint64_t az = uabs64(sz);
    u128 rhs = (u128)n_mu * (u128)n_mu * (u128)az * (u128)az;
    int m = 0;
    while (m + 1 < n_mu && (u128)(m + 1) * (u128)(m + 1) * (u128)d2 <= rhs) m++;
    return m;
}

static inline int mu_bin_mid(uint64_t d2, const int64_t s[3], const int64_t l[3], int n_mu) {
    int64_t p = s[0] * l[0] + s[1] * l[1] + s[2] * l[2];
    uint64_t q = (uint64_t)(l[0] * l[0]) + (uint64_t)(l[1] * l[1]) + (uint64_t)(l[2] * l[2]);
    if (d2 == 0 || q == 0) return 0;
    uint64_t ap = uabs64(p);
    u128 rhs = (u128)n_mu * (u128)n_mu * (u128)ap * (u128)ap;
    u128 dq = (u128)d2 * (u128)q;
    int m = 0;
    while (m + 1 < n_mu && (u128)(m + 1) * (u128)(m + 1) * dq <= rhs) m++;
    return m;
}

/*
 * a, b: SoA int32 coordinates, x[0..n) then y[0..n) then z[0..n).
 * box: periodic side in units (> 0, even), or 0 for open geometry.
 * los: 0 plane-parallel z, 1 midpoint, 2 (r_p, pi) along z with pi_max.
 * edges: n_r + 1 strictly increasing non-negative integers.
 * counts: uint64 [n_r][n_mu], overwritten.
 * n_threads <= 0: OpenMP default.  Returns the thread count used.
 */
int oracle_count_pairs(const int32_t* a, int64_t na, const int32_t* b, int64_t nb,
                       int auto_pairs, int64_t box, int los, int64_t pi_max,
                       int n_r, const int64_t* edges, int n_mu,
                       uint64_t* counts, int n_threads) {
    const int nbins = n_r * n_mu;
    uint64_t* e2 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n_r + 1));
    for (int k = 0; k <= n_r; k++) e2[k] = (uint64_t)(edges[k] * edges[k]);
    memset(counts, 0, sizeof(uint64_t) * (size_t)nbins);
    int used = 1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
        uint64_t* h = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < na; i++) {
            const int64_t xi[3] = {a[i], a[na + i], a[2 * na + i]};
            for (int64_t j = auto_pairs ? i + 1 : 0; j < nb; j++) {
                const int64_t xj[3] = {b[j], b[nb + j], b[2 * nb + j]};
                int64_t s[3];
                for (int c = 0; c < 3; c++) s[c] = wrap(xj[c] - xi[c], box);
                if (los == 2) {
                    const uint64_t rp2 = (uint64_t)(s[0] * s[0]) + (uint64_t)(s[1] * s[1]);
                    const int kp = r_bin(rp2, e2, n_r);
                    const uint64_t az = uabs64(s[2]);
                    if (kp < 0 || az >= (uint64_t)pi_max) continue;
                    h[kp * n_mu + (int)(((uint64_t)n_mu * az) / (uint64_t)pi_max)]++;
                    continue;
                }
                uint64_t d2 = (uint64_t)(s[0] * s[0]) + (uint64_t)(s[1] * s[1]) +
                              (uint64_t)(s[2] * s[2]);
                int k = r_bin(d2, e2, n_r);
                if (k < 0) continue;
                int m;
                if (los == 0) {
                    m = mu_bin_z(d2, s[2], n_mu);
                } else {
                    int64_t l[3];
                    for (int c = 0; c < 3; c++) l[c] = xi[c] + xj[c];
                    m = mu_bin_mid(d2, s, l, n_mu);
                }
                h[k * n_mu + m]++;
            }
        }
#pragma omp critical
        for (int t = 0; t < nbins; t++) counts[t] += h[t];
        free(h);
    }
    free(e2);
    return used;
}
