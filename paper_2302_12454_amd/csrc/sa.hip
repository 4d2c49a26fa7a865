// Traditional simulated annealing (serial single-spin Metropolis), the baseline of Section 4.4 and
// Table 4, as a many-chain kernel: one wave of 64 lanes runs one chain.
//
// A chain keeps its spins (int8, +-1) and its local fields F_j = sum_k J_jk sigma_k (int32) in LDS.
// Every cycle draws one Philox block (the same value in every lane), picks spin i, and evaluates the
// energy change of flipping it, dE = 2 sigma_i (h_i + F_i) (H of Eq. 1).  An accepted flip updates all
// fields from row i of J (J is symmetric: F_j += 2 sigma_i' J_ij) and the chain's energy by dE.  The
// acceptance test compares the 32-bit draw with 2^32 exp(-dE beta(t)) computed by sa_exp_neg, whose
// operation sequence is fixed (no contraction into fused multiply-adds), so that a host evaluation of
// the same function decides identically.
#include "internal.hpp"
#include "philox.hpp"

namespace ssqa {
namespace {

constexpr uint32_t kSAInitTag = 0xFFFFFFFEu;
constexpr uint32_t kSAStepTag = 0xFFFFFFFFu;
constexpr int kSAMaxWaves = 4;

constexpr double inv_factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;   // exact: 13! < 2^53
    return 1.0 / f;                        // rounded once
}

// J_ij from the P int8 planes of the fragment-tiled layout (J = sum_p 256^p J_p).
__device__ __forceinline__ int j_value(const DeviceProblem& prob, int i, int j) {
    const size_t off = tiled_offset(i, j, prob.np);
    const size_t plane = (size_t)prob.np * prob.np;
    int v = 0;
    for (int p = prob.planes - 1; p >= 0; --p) v = v * 256 + (int)prob.J[p * plane + off];
    return v;
}

__global__ __launch_bounds__(kSAMaxWaves * 64) void sa_kernel(SAArgs a) {
    extern __shared__ int32_t sa_lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b = blockIdx.x * (blockDim.x >> 6) + wave;
    if (b >= a.T) return;                    // whole wave: no workgroup barrier is used below
    const DeviceProblem& prob = a.prob;
    const int n = prob.n;
    const int stride = sa_lds_words(prob.np);
    int32_t* F = sa_lds + wave * stride;
    int8_t* s = reinterpret_cast<int8_t*>(F + prob.np);

    // initial spins: block (i >> 7, init tag, 0, b), spin i takes bit i & 31 of word (i & 127) >> 5
    for (int blk = lane; blk * 128 < n; blk += 64) {
        const Philox4 x = philox4x32_10((uint32_t)blk, kSAInitTag, 0u, (uint32_t)b, a.key0, a.key1);
        for (int o = 0; o < 128; ++o) {
            const int i = blk * 128 + o;
            if (i < n) s[i] = ((x.v[o >> 5] >> (o & 31)) & 1u) ? 1 : -1;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // fields and energy: H = -sum_j h_j s_j - (1/2) sum_j s_j F_j
    long long e_part = 0;
    for (int j = lane; j < n; j += 64) {
        int f = 0;
        for (int k = 0; k < n; ++k) f += j_value(prob, j, k) * (int)s[k];
        F[j] = f;
        e_part += (long long)s[j] * (2LL * prob.h[j] + f);
    }
    for (int off = 32; off >= 1; off >>= 1) e_part += __shfl_xor(e_part, off);
    long long e = -e_part / 2;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    long long best = e;
    int hit = (a.target != INT64_MIN && e == a.target) ? 0 : -1;
    if (a.trace && lane == 0) a.trace[b] = e;
    for (int t = 0; t < a.cycles; ++t) {
        const Philox4 x = philox4x32_10((uint32_t)t, kSAStepTag, 0u, (uint32_t)b, a.key0, a.key1);
        const uint32_t w0 = __builtin_amdgcn_readfirstlane(x.v[0]);
        const uint32_t w1 = __builtin_amdgcn_readfirstlane(x.v[1]);
        const int i = (int)(((uint64_t)w0 * (uint64_t)n) >> 32);
        const int si = __builtin_amdgcn_readfirstlane((int)s[i]);
        const int fi = __builtin_amdgcn_readfirstlane(F[i]);
        const long long de = 2LL * si * ((long long)prob.h[i] + fi);
        int accept = de <= 0;
        if (!accept) accept = __builtin_amdgcn_readfirstlane((double)w1 < sa_accept_threshold(de, a.beta[t]) ? 1 : 0);
        if (accept) {
            const int two_s = -2 * si;            // 2 sigma_i after the flip
            for (int j = lane; j < n; j += 64) F[j] += two_s * j_value(prob, i, j);
            if (lane == 0) s[i] = (int8_t)(-si);
            e += de;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (e < best) best = e;
        if (hit < 0 && a.target != INT64_MIN && e == a.target) hit = t + 1;
        if (a.trace && lane == 0) a.trace[(size_t)(t + 1) * a.T + b] = e;
    }
    if (lane == 0) {
        a.best[b] = best;
        a.first_hit[b] = hit;
        if (a.final_energy) a.final_energy[b] = e;
    }
    if (a.final_spins)
        for (int j = lane; j < n; j += 64) a.final_spins[(size_t)b * n + j] = s[j];
}

}  // namespace

// exp(-x) for x >= 0: n = floor(x / ln 2 + 1/2), r = n ln 2 - x, the degree-13 Taylor polynomial of
// exp(r) in Horner form, times 2^-n; 0 beyond x = 700 (every value stays a normal double).
__host__ __device__ double sa_exp_neg(double x) {
#pragma clang fp contract(off)
    constexpr double kLn2 = 0.6931471805599453;
    constexpr double kInvLn2 = 1.4426950408889634;
    if (x > 700.0) return 0.0;
    const double n = floor(x * kInvLn2 + 0.5);
    const double r = n * kLn2 - x;
    double p = inv_factorial(13);
    p = p * r + inv_factorial(12);
    p = p * r + inv_factorial(11);
    p = p * r + inv_factorial(10);
    p = p * r + inv_factorial(9);
    p = p * r + inv_factorial(8);
    p = p * r + inv_factorial(7);
    p = p * r + inv_factorial(6);
    p = p * r + inv_factorial(5);
    p = p * r + inv_factorial(4);
    p = p * r + inv_factorial(3);
    p = p * r + inv_factorial(2);
    p = p * r + inv_factorial(1);
    p = p * r + inv_factorial(0);
    return ldexp(p, -(int)n);
}

__host__ __device__ double sa_accept_threshold(long long de, double beta) {
#pragma clang fp contract(off)
    return ldexp(sa_exp_neg((double)de * beta), 32);
}

int sa_waves_per_group(int np) {
    const int per_wave = sa_lds_words(np) * 4;
    const int w = (160 * 1024) / per_wave;
    return w < 1 ? 0 : (w > kSAMaxWaves ? kSAMaxWaves : w);
}

}  // namespace ssqa

extern "C" double ssqa_sa_accept_threshold(int64_t de, double beta) { return ssqa::sa_accept_threshold(de, beta); }

namespace ssqa {

hipError_t launch_sa(const SAArgs& a, hipStream_t stream) {
    const int waves = sa_waves_per_group(a.prob.np);
    if (waves < 1) return hipErrorInvalidValue;
    const size_t lds = (size_t)waves * sa_lds_words(a.prob.np) * 4;
    static const hipError_t cfg =
        hipFuncSetAttribute(reinterpret_cast<const void*>(sa_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (cfg != hipSuccess) return cfg;
    const int groups = (a.T + waves - 1) / waves;
    hipLaunchKernelGGL(sa_kernel, dim3(groups), dim3(waves * 64), lds, stream, a);
    return hipGetLastError();
}

}  // namespace ssqa
