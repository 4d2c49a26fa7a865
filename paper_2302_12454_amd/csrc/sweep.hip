// SSQA sweep kernels for gfx950 (CDNA4).
//
// One cycle of SSQA (Section 3.2, Eq. 6a-c) updates every spin i of every replica k of every trial b
// from the state at cycle t.  The only O(N) term per spin is the field sum_j J_ij sigma_{j,k}(t); over
// all columns c = (b, k) it is the dense product F = J . Sigma (N x N by N x columns), computed here on
// int8 MFMA with int32 accumulation.  Everything else (noise, replica coupling, counter, sign, energy)
// is a fused integer epilogue on the accumulators.
//
// Design (trial-stationary persistent workgroups):
//  * A workgroup owns NB columns holding whole trials (the replica ring of Eq. 4 / Fig. 2 never leaves
//    the workgroup) and runs every cycle of a launch on its own: a cycle needs sigma(t) of all N spins of
//    the same columns only, so the per-cycle barrier is a workgroup barrier, never a grid barrier.
//  * sigma(t) lives in LDS as bit planes [column][N/32 words] (bit = 1 for +1).  A ring of d + 2 planes
//    holds sigma(t+1) (being written), sigma(t) (the MFMA operand) and sigma(t-1) .. sigma(t-d) (the
//    delayed coupling of Eq. 6a).  The counters Is stay in device memory as int8 [column][N].
//  * The MFMA runs on x = (sigma + 1) / 2 in {0, 1}: sum_j J_ij sigma_j = 2 sum_j J_ij x_j - sum_j J_ij.
//    16 bits of a bit plane expand to the 16 operand bytes of one lane with one multiply per 4 bytes.
//  * Each wave takes whole 128-row tiles (one Philox block of 128 spins per column) for all NB columns:
//    8 A fragments (rows, read from J in device memory) x NBF B fragments (columns, from LDS) per K
//    step of 64.  Rows are assigned to MFMA output slots so that lane group g of a 16 x 16 accumulator
//    holds the 32 consecutive rows 32 g .. 32 g + 31 of its column, i.e. exactly one 32-bit word of the
//    Philox block and of the bit plane.
//  * J with entries beyond int8 is split into P planes; the K loop runs once per plane, most
//    significant first, scaling the accumulator by 256 in between (exact Horner evaluation).

#include "internal.hpp"
#include "philox.hpp"

namespace ssqa {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = kWaves * 64;

// Columns per workgroup.
constexpr int kNBF = 4;              // 16-column MFMA fragments per workgroup
constexpr int kNB = 16 * kNBF;

__device__ __forceinline__ int plane_stride(int np) { return np / 32 + 1; }

// 16 bits (bit m = x for K offset m) -> 16 operand bytes 0/1 in K order.
__device__ __forceinline__ v4i expand16(uint32_t v) {
    v4i r;
    r[0] = (int)((((v >> 0) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[1] = (int)((((v >> 4) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[2] = (int)((((v >> 8) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[3] = (int)((((v >> 12) & 0xFu) * 0x00204081u) & 0x01010101u);
    return r;
}

__device__ __forceinline__ int sign_of_bit(uint32_t w, int m) { return ((w >> m) & 1u) ? 1 : -1; }

__device__ __forceinline__ int8_t get_byte(const v4i& v, int m) { return (int8_t)((v[m >> 2] >> (8 * (m & 3))) & 0xFF); }

__device__ __forceinline__ void put_byte(v4i& v, int m, int x) {
    const int sh = 8 * (m & 3);
    v[m >> 2] = (v[m >> 2] & ~(0xFF << sh)) | ((x & 0xFF) << sh);
}

__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepArgs a) {
    extern __shared__ uint32_t lds[];
    const int np = a.prob.np;
    const int n = a.prob.n;
    const int cstride = plane_stride(np);
    const int plane_words = kNB * cstride;
    const int npl = a.delay + 2;
    uint32_t* planes = lds;
    int32_t* e_acc = reinterpret_cast<int32_t*>(lds + npl * plane_words);      // [kNB]
    int32_t* hit_l = e_acc + kNB;                                               // [kNB]
    long long* best_l = reinterpret_cast<long long*>(hit_l + kNB);             // [kNB] (8-byte aligned)

    const int wg = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col16 = lane & 15;
    const int g = lane >> 4;
    const int ntiles = np / kTileRows;
    const int nsteps = np / kStepK;
    const int R = a.R;
    const int b0 = wg * a.tpw;
    const int words = np / 32;
    int8_t* is_wg = a.is_state + (size_t)wg * kNB * np;

    for (int c = tid; c < kNB; c += kThreads) e_acc[c] = 0;
    for (int lb = tid; lb < a.tpw; lb += kThreads) {
        const int b = b0 + lb;
        const bool fresh = (a.t_begin == 0);
        best_l[lb] = (b < a.T && !fresh) ? a.best[b] : INT64_MAX;
        hit_l[lb] = (b < a.T && !fresh) ? a.first_hit[b] : -1;
    }

    if (a.t_begin == 0) {
        // sigma(0) and Is(0) from the random stream, tag 0; sigma(-s) = sigma(0) for s = 1..d.
        for (int u = tid; u < ntiles * kNB; u += kThreads) {
            const int tile = u / kNB;
            const int c = u - tile * kNB;
            const int k = c % R;
            const int b = b0 + c / R;
            const Philox4 x = philox4x32_10(0u, (uint32_t)tile, (uint32_t)k, (uint32_t)b, a.key0, a.key1);
            for (int w = 0; w < 4; ++w) {
                for (int s = 0; s <= a.delay; ++s) {
                    const int p = (npl - s) % npl;
                    planes[p * plane_words + c * cstride + tile * 4 + w] = x.v[w];
                }
                v4i* dst = reinterpret_cast<v4i*>(is_wg + (size_t)c * np + tile * kTileRows + 32 * w);
                v4i lo = {0, 0, 0, 0}, hi = {0, 0, 0, 0};
                for (int m = 0; m < 32; ++m) {
                    const int val = ((x.v[w] >> m) & 1u) ? 0 : -a.alpha;
                    if (m < 16) put_byte(lo, m, val); else put_byte(hi, m - 16, val);
                }
                dst[0] = lo;
                dst[1] = hi;
            }
        }
    } else {
        // sigma(t_begin) = sign of the counters; sigma(t_begin - s) from the saved history.
        const int p_cur = a.t_begin % npl;
        for (int u = tid; u < kNB * words; u += kThreads) {
            const int c = u / words;
            const int w = u - c * words;
            const v4i* src = reinterpret_cast<const v4i*>(is_wg + (size_t)c * np + 32 * w);
            const v4i lo = src[0], hi = src[1];
            uint32_t bits = 0;
            for (int m = 0; m < 32; ++m) {
                const int8_t v = (m < 16) ? get_byte(lo, m) : get_byte(hi, m - 16);
                bits |= (uint32_t)(v >= 0) << m;
            }
            planes[p_cur * plane_words + c * cstride + w] = bits;
            for (int s = 1; s <= a.delay; ++s) {
                const int p = ((a.t_begin - s) % npl + npl) % npl;
                planes[p * plane_words + c * cstride + w] =
                    a.hist_state[(((size_t)wg * a.delay + (s - 1)) * kNB + c) * words + w];
            }
        }
    }
    __syncthreads();

    const int32_t* __restrict__ hvec = a.prob.h;
    const int32_t* __restrict__ rsum = a.prob.rowsum;
    const int P = a.prob.planes;

    for (int t = a.t_begin; t <= a.t_end; ++t) {
        const bool update = t < a.t_end;
        if (!update && !a.final_pass) break;
        const int p_cur = t % npl;
        const int p_next = (t + 1) % npl;
        const int p_del = (t - a.delay + npl) % npl;
        const int q = update ? a.jperp[t] : 0;
        const int i0 = update ? a.i0[t] : 0;
        const uint32_t* pl_cur = planes + p_cur * plane_words;

        for (int tile = wave; tile < ntiles; tile += kWaves) {
            v4i acc[8][kNBF];
#pragma unroll
            for (int ai = 0; ai < 8; ++ai)
#pragma unroll
                for (int f = 0; f < kNBF; ++f) acc[ai][f] = v4i{0, 0, 0, 0};

            // Row of J feeding output slot (ai, r = col16): tile row 32 (r / 4) + 4 ai + r % 4.
            const int row_base = tile * kTileRows + 32 * (col16 >> 2) + (col16 & 3);
            for (int p = P - 1; p >= 0; --p) {
                if (p < P - 1) {
#pragma unroll
                    for (int ai = 0; ai < 8; ++ai)
#pragma unroll
                        for (int f = 0; f < kNBF; ++f) acc[ai][f] = acc[ai][f] * 256;
                }
                const int8_t* Jp = a.prob.J + (size_t)p * np * np + (size_t)row_base * np + 16 * g;
                for (int s = 0; s < nsteps; ++s) {
                    v4i A[8];
#pragma unroll
                    for (int ai = 0; ai < 8; ++ai)
                        A[ai] = *reinterpret_cast<const v4i*>(Jp + (size_t)(4 * ai) * np + s * kStepK);
                    v4i B[kNBF];
                    const int wsel = 2 * s + (g >> 1);
                    const int sh = 16 * (g & 1);
#pragma unroll
                    for (int f = 0; f < kNBF; ++f) {
                        const uint32_t w = pl_cur[(16 * f + col16) * cstride + wsel];
                        B[f] = expand16((w >> sh) & 0xFFFFu);
                    }
#pragma unroll
                    for (int ai = 0; ai < 8; ++ai)
#pragma unroll
                        for (int f = 0; f < kNBF; ++f)
                            acc[ai][f] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[ai], B[f], acc[ai][f], 0, 0, 0);
                }
            }

            // Fused epilogue: lane (column 16 f + col16, group g) owns rows tile*128 + 32 g + 0..31.
            const int word = tile * 4 + g;
            const int row0 = tile * kTileRows + 32 * g;
#pragma unroll
            for (int f = 0; f < kNBF; ++f) {
                const int c = 16 * f + col16;
                const int lb = c / R;
                const int k = c - lb * R;
                const int b = b0 + lb;
                const bool valid = (c < a.cols_wg) && (b < a.T);
                const uint32_t sig_w = pl_cur[c * cstride + word];
                uint32_t up_w = 0, dn_w = 0, noise_w = 0;
                v4i is_lo = {0, 0, 0, 0}, is_hi = {0, 0, 0, 0};
                v4i* is_ptr = reinterpret_cast<v4i*>(is_wg + (size_t)c * np + row0);
                if (update) {
                    const int c_up = valid ? lb * R + (k + 1 == R ? 0 : k + 1) : c;
                    const int c_dn = valid ? lb * R + (k == 0 ? R - 1 : k - 1) : c;
                    up_w = planes[p_del * plane_words + c_up * cstride + word];
                    dn_w = planes[p_del * plane_words + c_dn * cstride + word];
                    noise_w = philox4x32_10((uint32_t)(t + 1), (uint32_t)tile, (uint32_t)k, (uint32_t)b,
                                            a.key0, a.key1).v[g];
                    is_lo = is_ptr[0];
                    is_hi = is_ptr[1];
                }
                int epart = 0;
                uint32_t new_w = 0;
#pragma unroll
                for (int ai = 0; ai < 8; ++ai) {
                    const v4i h4 = *reinterpret_cast<const v4i*>(hvec + row0 + 4 * ai);
                    const v4i r4 = *reinterpret_cast<const v4i*>(rsum + row0 + 4 * ai);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int m = 4 * ai + j;
                        const int i = row0 + m;
                        const int F = 2 * acc[ai][f][j] - r4[j];
                        const int si = sign_of_bit(sig_w, m);
                        if (i < n) epart += si * (2 * h4[j] + F);
                        if (update) {
                            int coupling = q * sign_of_bit(up_w, m);
                            if (a.mode == 1) coupling += q * sign_of_bit(dn_w, m);
                            const int isv = (m < 16) ? get_byte(is_lo, m) : get_byte(is_hi, m - 16);
                            const int sum = isv + h4[j] + F + a.noise_amp * sign_of_bit(noise_w, m) + coupling;
                            const int nv = sum >= i0 ? i0 - a.alpha : (sum < -i0 ? -i0 : sum);
                            if (m < 16) put_byte(is_lo, m, nv); else put_byte(is_hi, m - 16, nv);
                            new_w |= (uint32_t)(nv >= 0) << m;
                        }
                    }
                }
                if (update) {
                    is_ptr[0] = is_lo;
                    is_ptr[1] = is_hi;
                    planes[p_next * plane_words + c * cstride + word] = new_w;
                }
                epart += __shfl_xor(epart, 16);
                epart += __shfl_xor(epart, 32);
                if (g == 0 && valid) atomicAdd(&e_acc[c], epart);
            }
        }
        __syncthreads();

        // H_p of every replica at cycle t: sum_i sigma_i (2 h_i + F_i) = -2 H_p.
        if (a.trace) {
            for (int c = tid; c < a.cols_wg; c += kThreads) {
                const int lb = c / R;
                const int b = b0 + lb;
                if (b < a.T) a.trace[(size_t)t * a.T * R + (size_t)b * R + (c - lb * R)] = -e_acc[c] / 2;
            }
        }
        for (int lb = tid; lb < a.tpw; lb += kThreads) {
            const int b = b0 + lb;
            if (b >= a.T) continue;
            long long m = INT64_MAX;
            for (int k = 0; k < R; ++k) {
                const long long e = -(long long)e_acc[lb * R + k] / 2;
                m = e < m ? e : m;
            }
            if (m < best_l[lb]) best_l[lb] = m;
            if (hit_l[lb] < 0 && a.target != INT64_MIN && m == a.target) hit_l[lb] = t;
        }
        __syncthreads();
        for (int c = tid; c < kNB; c += kThreads) e_acc[c] = 0;
        __syncthreads();
    }

    for (int lb = tid; lb < a.tpw; lb += kThreads) {
        const int b = b0 + lb;
        if (b < a.T) {
            a.best[b] = best_l[lb];
            a.first_hit[b] = hit_l[lb];
        }
    }
    if (!a.final_pass && a.delay > 0) {
        for (int u = tid; u < kNB * words; u += kThreads) {
            const int c = u / words;
            const int w = u - c * words;
            for (int s = 1; s <= a.delay; ++s) {
                const int p = ((a.t_end - s) % npl + npl) % npl;
                a.hist_state[(((size_t)wg * a.delay + (s - 1)) * kNB + c) * words + w] =
                    planes[p * plane_words + c * cstride + w];
            }
        }
    }
}

// int32 J [n][n] -> P balanced int8 planes [P][np][np] (J = sum_p 256^p J_p), zero padded;
// also the padded h and the row sums of J.
__global__ void prepare_planes_kernel(const int32_t* J32, const int32_t* h32, int32_t n, int32_t np,
                                      int32_t P, int8_t* Jp, int32_t* h_pad, int32_t* rowsum) {
    const int i = blockIdx.x;
    if (i >= np) return;
    long long rs = 0;
    for (int j = threadIdx.x; j < np; j += blockDim.x) {
        int v = (i < n && j < n) ? J32[(size_t)i * n + j] : 0;
        rs += v;
        for (int p = 0; p < P; ++p) {
            const int8_t d = (int8_t)(v & 0xFF);
            Jp[(size_t)p * np * np + (size_t)i * np + j] = d;
            v = (v - d) >> 8;
        }
    }
    __shared__ long long part[256];
    part[threadIdx.x] = rs;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rowsum[i] = (int32_t)part[0];
        h_pad[i] = i < n ? h32[i] : 0;
    }
}

__global__ void copy_final_is_kernel(const int8_t* is_state, int32_t np, int32_t n, int32_t R, int32_t T,
                                     int32_t tpw, int8_t* out) {
    const int col = blockIdx.x;   // b * R + k
    const int b = col / R;
    const int k = col - b * R;
    if (b >= T) return;
    const int wg = b / tpw;
    const int lc = (b - wg * tpw) * R + k;
    const int8_t* src = is_state + ((size_t)wg * kNB + lc) * np;
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[(size_t)col * n + i] = src[i];
}

// H_p of explicit +-1 configurations: one workgroup per configuration, J read plane by plane.
__global__ void energy_kernel(DeviceProblem prob, const int8_t* spins, int32_t cols, int64_t* energies) {
    const int c = blockIdx.x;
    if (c >= cols) return;
    const int8_t* s = spins + (size_t)c * prob.n;
    long long part = 0;
    for (int i = threadIdx.x; i < prob.n; i += blockDim.x) {
        long long F = 0;
        for (int p = prob.planes - 1; p >= 0; --p) {
            const int8_t* row = prob.J + (size_t)p * prob.np * prob.np + (size_t)i * prob.np;
            long long acc = 0;
            for (int j = 0; j < prob.n; ++j) acc += (int)row[j] * (int)s[j];
            F = F * 256 + acc;
        }
        part += (long long)s[i] * (2LL * prob.h[i] + F);
    }
    __shared__ long long red[256];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) energies[c] = -red[0] / 2;
}

}  // namespace

int sweep_columns_per_wg() { return kNB; }

size_t sweep_lds_bytes(int np, int delay) {
    const size_t plane_words = (size_t)kNB * (np / 32 + 1);
    return (size_t)(delay + 2) * plane_words * 4 + (size_t)kNB * 4 * 2 + (size_t)kNB * 8 + 8;
}

hipError_t launch_prepare_planes(const int32_t* J32, const int32_t* h32, int32_t n, int32_t np, int32_t planes,
                                 int8_t* Jp, int32_t* h_pad, int32_t* rowsum, hipStream_t stream) {
    hipLaunchKernelGGL(prepare_planes_kernel, dim3(np), dim3(256), 0, stream, J32, h32, n, np, planes, Jp, h_pad,
                       rowsum);
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs& args, int n_wg, hipStream_t stream) {
    const size_t lds = sweep_lds_bytes(args.prob.np, args.delay);
    static bool configured = false;
    if (!configured) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        configured = true;
    }
    hipLaunchKernelGGL(sweep_kernel, dim3(n_wg), dim3(kThreads), lds, stream, args);
    return hipGetLastError();
}

hipError_t launch_copy_final_is(const int8_t* is_state, int32_t np, int32_t n, int32_t R, int32_t T, int32_t tpw,
                                int8_t* out, hipStream_t stream) {
    hipLaunchKernelGGL(copy_final_is_kernel, dim3(T * R), dim3(256), 0, stream, is_state, np, n, R, T, tpw, out);
    return hipGetLastError();
}

hipError_t launch_energy(const DeviceProblem& prob, const int8_t* spins, int32_t cols, int64_t* energies,
                         hipStream_t stream) {
    hipLaunchKernelGGL(energy_kernel, dim3(cols), dim3(256), 0, stream, prob, spins, cols, energies);
    return hipGetLastError();
}

}  // namespace ssqa
