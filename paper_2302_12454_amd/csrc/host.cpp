// Host helpers of the C ABI: annealing schedules and the graph-isomorphism mapping (see include/ssqa.h).
#include <stdint.h>

#include <cstdlib>
#include <vector>

#include "ssqa.h"

extern "C" {

// Section 4.2 / Table 2: iteration of tau * (beta + 1) cycles, J_perp raised by (jmax - jmin) / beta
// every tau cycles, reset at the start of every iteration.  Level l in [0, beta] is
// jmin + l (jmax - jmin) / beta; scaled by S it must be an integer.
ssqa_status ssqa_jperp_schedule(int32_t cycles, int32_t tau, int32_t beta, int32_t jmin_num, int32_t jmax_num,
                                int32_t den, int32_t scale, int32_t* out) {
    if (cycles < 0 || tau < 1 || beta < 1 || den < 1 || scale < 1 || (cycles > 0 && !out)) return SSQA_EINVAL;
    // scale * (jmin + l (jmax - jmin) / beta) = scale (beta jmin_num + l (jmax_num - jmin_num)) / (beta den)
    std::vector<int32_t> level(beta + 1);
    for (int l = 0; l <= beta; ++l) {
        const long long num = (long long)scale * ((long long)beta * jmin_num + (long long)l * (jmax_num - jmin_num));
        const long long d = (long long)beta * den;
        if (num % d != 0) return SSQA_EINVAL;
        level[l] = (int32_t)(num / d);
    }
    const int period = tau * (beta + 1);
    for (int t = 0; t < cycles; ++t) out[t] = level[(t % period) / tau];
    return SSQA_OK;
}

// Section 4.4 (SA): 1/T(t+1) = 1/T(t) + Delta every cycle, from t_start at t = 0 to t_end at the last
// cycle; beta(t) = 1/(scale T(t)) = b0 + t Delta, each value from one product and one sum.
ssqa_status ssqa_sa_schedule(int32_t cycles, double t_start, double t_end, int32_t scale, double* beta) {
#pragma clang fp contract(off)
    if (cycles < 1 || scale < 1 || !beta || !(t_start > 0.0) || !(t_end > 0.0)) return SSQA_EINVAL;
    const double b0 = 1.0 / ((double)scale * t_start);
    const double b1 = 1.0 / ((double)scale * t_end);
    if (cycles == 1) {
        beta[0] = b0;
        return SSQA_OK;
    }
    const double delta = (b1 - b0) / (double)(cycles - 1);
    for (int t = 0; t < cycles; ++t) beta[t] = b0 + (double)t * delta;
    return SSQA_OK;
}

// Section 4.4: I_0 from i0_min multiplied by growth every tau cycles until i0_max, tau cycles at
// i0_max, then again from i0_min.
ssqa_status ssqa_ssa_i0_schedule(int32_t cycles, int32_t tau, int32_t growth, int32_t i0_min, int32_t i0_max,
                                 int32_t scale, int32_t* out) {
    if (cycles < 0 || tau < 1 || growth < 2 || i0_min < 1 || i0_max < i0_min || scale < 1 || (cycles > 0 && !out))
        return SSQA_EINVAL;
    std::vector<int32_t> level;
    for (long long v = i0_min;; v *= growth) {
        if (v >= i0_max) {
            level.push_back(i0_max);
            break;
        }
        level.push_back((int32_t)v);
    }
    const int period = tau * (int)level.size();
    for (int t = 0; t < cycles; ++t) {
        const long long v = (long long)scale * level[(t % period) / tau];
        if (v > INT32_MAX) return SSQA_ERANGE;
        out[t] = (int32_t)v;
    }
    return SSQA_OK;
}

// Section 4.1 (Eq. 8) and the QUBO-to-Ising mapping of Section 4.2 at integer scale S.
ssqa_status ssqa_gi_to_ising(int32_t n, const uint8_t* a1, const uint8_t* a2, int32_t c1, int32_t c2, int32_t scale,
                             int32_t* h, int32_t* J, int64_t* e_star) {
    if (n < 1 || n > 128 || !a1 || !a2 || !h || !J || !e_star || scale < 4 || scale % 4 != 0) return SSQA_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (a1[i * n + i] || a2[i * n + i]) return SSQA_EINVAL;
        for (int j = 0; j < n; ++j)
            if ((a1[i * n + j] != 0) != (a1[j * n + i] != 0) || (a2[i * n + j] != 0) != (a2[j * n + i] != 0))
                return SSQA_EINVAL;
    }
    const int N = n * n;
    const long long q4 = scale / 4, q2 = scale / 2;
    long long diag_sum = 0, upper_sum = 0;
    for (int p = 0; p < N; ++p) {
        const int u = p / n, i = p % n;
        long long row = 0;  // sum over q != p of Q_pq (upper triangle mirrored)
        for (int q = 0; q < N; ++q) {
            if (q == p) {
                J[(size_t)p * N + q] = 0;
                continue;
            }
            const int v = q / n, j = q % n;
            long long Q = 0;
            const bool su = (u == v), si = (i == j);
            if (su != si) {
                Q = 2LL * c1;
            } else if (!su && !si && ((a1[i * n + j] != 0) != (a2[u * n + v] != 0))) {
                Q = c2;
            }
            row += Q;
            if (q > p) upper_sum += Q;
            const long long Jv = -q4 * Q;
            if (Jv < INT32_MIN || Jv > INT32_MAX) return SSQA_ERANGE;
            J[(size_t)p * N + q] = (int32_t)Jv;
        }
        const long long Qpp = -2LL * c1;
        diag_sum += Qpp;
        const long long hv = -q2 * Qpp - q4 * row;
        if (hv < INT32_MIN || hv > INT32_MAX) return SSQA_ERANGE;
        h[p] = (int32_t)hv;
    }
    // S H_QUBO(x) = E(sigma) + S c with S c = (S/2) sum Q_pp + (S/4) sum_{p<q} Q_pq; at an isomorphism
    // Eq. 8 vanishes, i.e. H_QUBO = -2 n C1.
    const long long c_scaled = q2 * diag_sum + q4 * upper_sum;
    *e_star = -(long long)scale * 2LL * n * c1 - c_scaled;
    return SSQA_OK;
}

}  // extern "C"
