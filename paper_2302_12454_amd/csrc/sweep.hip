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

#include <mutex>
#include <type_traits>

#include "internal.hpp"
#include "philox.hpp"

namespace ssqa {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = kWaves * 64;

// Columns per workgroup: kNBF MFMA column fragments of 16 (kNBF = 4: 64 columns, the default; kNBF = 2:
// 32 columns, for large N where the bit planes of 64 columns would not fit in LDS; kNBF = 8: 128 columns with
// fp4 operands, one workgroup per CU and one wave per SIMD, whose 512 registers hold the 256 accumulators:
// each J fragment then feeds twice as many MFMAs).

__device__ __forceinline__ int plane_stride(int np) { return np / 32 + 1; }

// Bit-plane word layout.  Word w of a column holds spins 32 w .. 32 w + 31; spin offset
// o = 16 h + 4 j + m (h < 2, j < 4, m < 4) sits at bit 8 m + 4 h + j.  With this spread order the
// 16 MFMA operand bytes of a lane are (word >> (4 h + j)) & 0x01010101 for j = 0..3.
__host__ __device__ constexpr int bitpos(int o) { return 8 * (o & 3) + 4 * (o >> 4) + ((o >> 2) & 3); }

__device__ inline uint32_t spread_bits(uint32_t natural) {
    uint32_t r = 0;
    for (int o = 0; o < 32; ++o) r |= ((natural >> o) & 1u) << bitpos(o);
    return r;
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));

// fp4 (e2m1) operand of x = (sigma + 1) / 2 from one bit-plane word: 1.0 is nibble 0b0010.  Dword d takes
// the bits at positions congruent to d modulo 4, one per nibble (see tiled_offset_fp4 for the matching J).
__device__ __forceinline__ v4i expand_operand_fp4(uint32_t w) {
    v4i r;
    r[0] = (int)((w << 1) & 0x22222222u);
    r[1] = (int)(w & 0x22222222u);
    r[2] = (int)((w >> 1) & 0x22222222u);
    r[3] = (int)((w >> 2) & 0x22222222u);
    return r;
}

__device__ __forceinline__ v8i widen(const v4i& x) { return __builtin_shufflevector(x, x, 0, 1, 2, 3, -1, -1, -1, -1); }

__device__ __forceinline__ v4i expand_operand(uint32_t w) {
    // w already shifted by 4 h; bytes are 2 x = sigma + 1 in {0, 2}, so that the int32 accumulator collects
    // 2 sum_j J_ij x_j directly (as the fp4 product does through its scale)
    v4i r;
    r[0] = (int)((w << 1) & 0x02020202u);
    r[1] = (int)(w & 0x02020202u);
    r[2] = (int)((w >> 1) & 0x02020202u);
    r[3] = (int)((w >> 2) & 0x02020202u);
    return r;
}

// 16 bytes of J at byte offset voffset + soffset of the plane buffer.
__device__ __forceinline__ v4i load_j(__amdgpu_buffer_rsrc_t rsrc, int voffset, int soffset) {
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    const v4u x = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voffset, soffset, 0);
    return (v4i)x;
}

__device__ __forceinline__ int bfe_i(int w, int off, int width) { return __builtin_amdgcn_sbfe(w, off, width); }
__device__ __forceinline__ uint32_t bfe_u(uint32_t w, int off, int width) { return __builtin_amdgcn_ubfe(w, off, width); }

// The 8 A fragments (one K step of a 128-row tile) at byte offset `off` of the J buffer.
__device__ __forceinline__ void load_fragments(v4i (&A)[8], __amdgpu_buffer_rsrc_t rsrc, int voff, int off) {
#pragma unroll
    for (int ai = 0; ai < 8; ++ai) A[ai] = load_j(rsrc, voff, off + ai * 1024);
}

// One K step on int8 operands, column fragment by column fragment, as the fp4 step below: while the 8 MFMAs
// of fragment f run, the operand of fragment f + 1 (with kNext, after the last fragment, that of the next
// step's fragment 0 from `next0`) is expanded in their shadow, one VALU instruction after each MFMA.  With
// kReload, A[ai] is refilled from byte offset `next` right behind its last MFMA.  `bsh` selects the lane's
// half of each word.
template <int kNBF, bool kReload, bool kNext>
__device__ __forceinline__ void mma_i8_cols(v4i (&A)[8], v4i& Bc, const uint32_t (&cur)[kNBF], uint32_t next0, int bsh,
                                            v4i (&acc)[8][kNBF], __amdgpu_buffer_rsrc_t rsrc, int voff, int next) {
#pragma unroll
    for (int f = 0; f < kNBF; ++f) {
        v4i Bn = Bc;
        if (f + 1 < kNBF) Bn = expand_operand(cur[f + 1] >> bsh);
        else if (kNext) Bn = expand_operand(next0 >> bsh);
#pragma unroll
        for (int ai = 0; ai < 8; ++ai) {
            acc[ai][f] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[ai], Bc, acc[ai][f], 0, 0, 0);
            if (kReload && f == kNBF - 1) A[ai] = load_j(rsrc, voff, next + ai * 1024);
        }
#pragma unroll
        for (int ai = 0; ai < 8; ++ai) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);  // then one VALU instruction
            if (kReload && f == kNBF - 1) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // and one J load
        }
        __builtin_amdgcn_sched_barrier(0);
        Bc = Bn;
    }
}

// One fp4 (e2m1) MFMA, fp32 accumulation; J is scaled by 2 (e8m0 scale 128), x by 1.
__device__ __forceinline__ v4f mfma_fp4(const v4i& a, const v4i& b, const v4f& c) {
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(widen(a), widen(b), c, 4, 4, 0, 128, 0, 127);
}

// One K step on fp4 operands, column fragment by column fragment.  On entry Bc holds the expanded operand of
// fragment 0; cur[f] is the bit-plane word of fragment f.  While the 8 MFMAs of fragment f run, the operand of
// fragment f + 1 (with kNext, after the last fragment, that of the next step's fragment 0 from `next0`) is
// expanded in their shadow: an fp4 MFMA leaves the SIMD's issue port free for about one VALU instruction, so
// interleaved one by one the expansion costs almost nothing, while issued as a block it stalls the MFMAs.
// With kReload, A[ai] is refilled from byte offset `next` right behind its last MFMA.
template <int kNBF, bool kReload, bool kNext>
__device__ __forceinline__ void mma_fp4_cols(v4i (&A)[8], v4i& Bc, const uint32_t (&cur)[kNBF], uint32_t next0,
                                             v4f (&acc)[8][kNBF], __amdgpu_buffer_rsrc_t rsrc, int voff, int next) {
#pragma unroll
    for (int f = 0; f < kNBF; ++f) {
        v4i Bn = Bc;
        if (f + 1 < kNBF) Bn = expand_operand_fp4(cur[f + 1]);
        else if (kNext) Bn = expand_operand_fp4(next0);
#pragma unroll
        for (int ai = 0; ai < 8; ++ai) {
            acc[ai][f] = mfma_fp4(A[ai], Bc, acc[ai][f]);
            if (kReload && f == kNBF - 1) A[ai] = load_j(rsrc, voff, next + ai * 1024);
        }
#pragma unroll
        for (int ai = 0; ai < 8; ++ai) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);  // then one VALU instruction
            if (kReload && f == kNBF - 1) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // and one J load
        }
        __builtin_amdgcn_sched_barrier(0);
        Bc = Bn;
    }
}

typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v16i __attribute__((ext_vector_type(16)));

// One fp4 (e2m1) 32 x 32 x 64 MFMA, fp32 accumulation, J scaled by 2 and x by 1 as in mfma_fp4.  The 128- and
// 64-column blocks use it: an fp4 MFMA of this shape leaves the SIMD's issue port free for a few simple VALU
// instructions of the same wave (a 16 x 16 x 128 one, half its work, for about one), so the operand expansion
// and the interleaved loads cost the K loop nothing.
__device__ __forceinline__ v16f mfma_fp4_32(const v4i& a, const v4i& b, const v16f& c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(widen(a), widen(b), c, 4, 4, 0, 128, 0, 127);
}

// One K step (128) of a 128-row tile on 32 x 32 x 64 MFMAs, kNCB column blocks of 32.  A[kh][rb] is the J
// operand of row block rb for K half kh, cur[kh][cb] the bit-plane word of column block cb for K half kh.  On
// entry Bc holds the expanded operand of (kh, cb) = (0, 0); while the four MFMAs of one (kh, cb) run, the next
// operand is expanded in their shadow (with kNext, after the last one, the next step's first from `next0`).
// With kReload, A[kh][rb] is refilled from byte offset `next` right behind its last MFMA, half a step earlier
// for K half 0 than for K half 1.  With kStart the accumulators of K half 0 start from start[rb].
template <int kNCB, bool kReload, bool kNext, bool kStart>
__device__ __forceinline__ void mma_fp4_wide(v4i (&A)[2][4], v4i& Bc, const uint32_t (&cur)[2][kNCB], uint32_t next0,
                                             v16f (&acc)[4][kNCB], const v16f (&start)[4],
                                             __amdgpu_buffer_rsrc_t rsrc, int voff, int next) {
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
#pragma unroll
        for (int cb = 0; cb < kNCB; ++cb) {
            v4i Bn = Bc;
            if (cb + 1 < kNCB) Bn = expand_operand_fp4(cur[kh][cb + 1]);
            else if (kh == 0) Bn = expand_operand_fp4(cur[1][0]);
            else if (kNext) Bn = expand_operand_fp4(next0);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb][cb] = mfma_fp4_32(A[kh][rb], Bc, (kStart && kh == 0) ? start[rb] : acc[rb][cb]);
                if (kReload && cb == kNCB - 1) A[kh][rb] = load_j(rsrc, voff, next + rb * 2048 + kh * 512);
            }
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // then up to two VALU instructions
                if (kReload && cb == kNCB - 1) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // and one J load
            }
            __builtin_amdgcn_sched_barrier(0);
            Bc = Bn;
        }
    }
}

// The 32 int8 counters of this lane in column fragment f (column 16 f + lane % 16).  With fp4 operands they
// are read through the caches: the fp4 copy of J leaves room in L2, a one-wave-per-SIMD epilogue has no other
// wave to cover their latency, and streaming (nontemporal) loads of them measured 3-5 % slower on the whole
// anneal.  With int8 operands on 16 x 16 tiles J alone overflows L2, and cached counter loads evict it (3 %
// slower), so they stream.  On 32 x 32 tiles a unit reads half of a 128-byte counter line and the next unit
// the other half; streamed, each half fetched the line again and the int8 epilogue took twice as long, so
// there they go through the caches with either operand type.  The epilogue writes the counters back with
// streaming stores, which nothing reads before the next cycle.
template <bool kFp4>
__device__ __forceinline__ void load_counters(v4i (&c)[2], const int8_t* is_lane, int np, int f) {
    const v4i* src = reinterpret_cast<const v4i*>(is_lane + (size_t)16 * f * np);
    if constexpr (kFp4) {
        c[0] = src[0];
        c[1] = src[1];
    } else {
        c[0] = __builtin_nontemporal_load(src);
        c[1] = __builtin_nontemporal_load(src + 1);
    }
}

// One K step (64) of a 128-row tile on int8 32 x 32 x 32 MFMAs (single-plane J), as mma_fp4_wide: A[kh][rb] is
// the J operand of row block rb for K half kh (32), cur[kh][cb] the bit-plane word of column block cb for that
// half, whose lane half `bsh` holds the lane's 16 K values.
template <int kNCB, bool kReload, bool kNext>
__device__ __forceinline__ void mma_i8_wide(v4i (&A)[2][4], v4i& Bc, const uint32_t (&cur)[2][kNCB], uint32_t next0,
                                            int bsh, v16i (&acc)[4][kNCB], __amdgpu_buffer_rsrc_t rsrc, int voff,
                                            int next) {
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
#pragma unroll
        for (int cb = 0; cb < kNCB; ++cb) {
            v4i Bn = Bc;
            if (cb + 1 < kNCB) Bn = expand_operand(cur[kh][cb + 1] >> bsh);
            else if (kh == 0) Bn = expand_operand(cur[1][0] >> bsh);
            else if (kNext) Bn = expand_operand(next0 >> bsh);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[kh][rb], Bc, acc[rb][cb], 0, 0, 0);
                if (kReload && cb == kNCB - 1) A[kh][rb] = load_j(rsrc, voff, next + rb * 2048 + kh * 512);
            }
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // then up to two VALU instructions
                if (kReload && cb == kNCB - 1) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // and one J load
            }
            __builtin_amdgcn_sched_barrier(0);
            Bc = Bn;
        }
    }
}

template <bool kFp4>
__device__ __forceinline__ void load_counters_at(v4i (&c)[2], const int8_t* p) {
    const v4i* src = reinterpret_cast<const v4i*>(p);
    if constexpr (kFp4) {
        c[0] = src[0];
        c[1] = src[1];
    } else {
        c[0] = __builtin_nontemporal_load(src);
        c[1] = __builtin_nontemporal_load(src + 1);
    }
}

// Counters are fetched cnt_ahead fragments (units) ahead of their use: those of units 0 .. cnt_ahead - 1
// during the last K steps, that of unit u + cnt_ahead while the epilogue works on unit u (two with cached
// loads, where the deeper prefetch paid; one with streaming loads).  kCached: fp4 operands, or 32 x 32 tiles.
template <bool kCached>
constexpr int cnt_ahead() { return kCached ? 2 : 1; }

template <int kNBF, bool kFp4>
__device__ __forceinline__ void prefetch_counters(v4i (&cnt)[kNBF][2], const int8_t* is_lane, int np) {
#pragma unroll
    for (int f = 0; f < kNBF && f < cnt_ahead<kFp4>(); ++f) load_counters<kFp4>(cnt[f], is_lane, np, f);
}

// 4 rows of the tile's row vectors: lane l < 32 takes h - rowsum at rows 4 l .. 4 l + 3, lane l >= 32 takes h
// at rows 4 (l - 32) .. 4 (l - 32) + 3.
__device__ __forceinline__ v4i fetch_rows(const DeviceProblem& prob, int tile) {
    int ln = threadIdx.x & 63;
    asm volatile("" : "+v"(ln));
    return *reinterpret_cast<const v4i*>((ln < 32 ? prob.hr : prob.h) + tile * kTileRows + 4 * (ln & 31));
}

// Writes the row vectors fetched by this lane into the wave's staging area, each plus its cycle constant.
// The lane index is laundered so that no per-lane select is hoisted out of the tile loop into registers.
__device__ __forceinline__ void stage_rows(int32_t* st, v4i rowv, int add_h, int add_e) {
    int ln = threadIdx.x & 63;
    asm volatile("" : "+v"(ln));
    const int add = ln < 32 ? add_h : add_e;
    rowv += add;
    *reinterpret_cast<v4i*>(st + 4 * ln) = rowv;
}

struct EpilogueCtx {
    const uint32_t* pl_cur;   // sigma(t) bit plane
    const uint32_t* pl_del;   // sigma(t - d) bit plane
    uint32_t* pl_next;        // sigma(t + 1) bit plane
    const uint32_t* noise_lds;
    const uint32_t* colinfo;
    int32_t* e_acc;
    int8_t* is_wg;
    // This wave's staged row constants: [0, 128) the per-row part of the counter input, [128, 256) the
    // per-row part of the energy term (see sweep_block for what each holds).
    const int32_t* rows;
    int np, cstride, tile, wave, lane;
    // sigma(t - d) and sigma(t + 1): word w of column c at c * cstride_dn + w - dn_off (the whole plane, or in the
    // row-split form the group's rows only)
    int cstride_dn, dn_off;
    int coff;                 // first column of the fragments this call covers (0, or 64 for a column half)
    int ncols;                // columns per wave in the noise area (the block width)
    int two_n, two_q, i0, alpha;
    uint32_t qflip;           // fast path: 0, or all ones when J_perp < 0 (the coupling bits are complemented)
};

__device__ __forceinline__ int med3_i32(int x, int lo, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// (a ^ b) + c in one instruction.
__device__ __forceinline__ int xad_u32(int a, int b, int c) {
    int r;
    asm("v_xad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Bits 4 a .. 4 a + 3 of w, one per byte (bit 4 a + j -> bit 8 j).
__device__ __forceinline__ uint32_t nibble_to_bytes(uint32_t w, int a) {
    return (bfe_u(w, 4 * a, 4) * 0x00204081u) & 0x01010101u;
}

// An accumulator value read out of its AGPR where it is used (128-column blocks, whose 256 accumulators live
// in AGPRs).  Without it the register allocator copies most accumulators to VGPRs during the last K step,
// which exceeds the VALU slots the MFMAs leave free there and crowds the epilogue into spilling; with it the
// kernel needs no scratch and the anneal measured 2 % faster.
__device__ __forceinline__ int agpr_read(int x) {
    int r;
    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(r) : "a"(x));
    return r;
}

// Accumulator (row offset 4 ai + j of unit u) in the two MFMA output layouts: 16 x 16 tiles (acc[ai][u], unit u
// = column fragment u) and 32 x 32 tiles (acc[rb][cb], unit u = (cb, rr) = (u / 2, u % 2), whose register
// 4 i + j holds tile row 64 (i & 1) + 32 (lane / 32) + 8 rb + 4 (i >> 1) + j).  kAgpr reads it out of its AGPR
// where it is used.
template <bool kAgpr, int kN>
__device__ __forceinline__ int acc_value(const v4i (&acc)[8][kN], int u, int ai, int j) {
    return kAgpr ? agpr_read(acc[ai][u][j]) : acc[ai][u][j];
}
template <bool kAgpr, int kN>
__device__ __forceinline__ int acc_value(const v16i (&acc)[4][kN], int u, int ai, int j) {
    const int v = acc[ai >> 1][u >> 1][4 * (2 * (ai & 1) + (u & 1)) + j];
    return kAgpr ? agpr_read(v) : v;
}

// Fused epilogue of one 128-row tile for the kUnits units of this wave.  A unit is one column and one run of
// 32 consecutive tile rows of it: with 16 x 16 MFMA tiles (kWide false) unit u is column 16 u + lane % 16 and
// run lane / 16 (tile rows 32 (lane / 16) ..); with 32 x 32 tiles (kWide) unit u = 2 cb + rr is column
// 32 cb + lane % 32 and run 2 rr + lane / 32, so that the two units of a column, whose counters share the
// tile's 128-byte line, follow each other (their stores then meet in L2 and leave as whole lines; with the
// column's halves kNCB units apart they left partly as halves: 28 % more HBM write traffic).  The lane owns one 32-bit word of every bit plane and of the
// Philox block in each unit, and 32 consecutive int8 counters.  With kUpdate the counters and the next bit
// plane are written (Eq. 6a-c); the energy sum_i sigma_i (2 h_i + F_i) of the current state is always
// accumulated.
//
// Row offset o = 4 a + j of a run sits in byte j of counter dword a and at bit 8 j + a of the bit-plane words
// (bitpos), and at bit o of the Philox word.
//
// kFast (alpha = 1, and max_t I_0 + 2 n_rnd + 2 max_t |J_perp| (1 + mode) <= 128): the counters of the 4
// rows of dword a, offset by 128, and their noise and coupling increments 2 n_rnd [r = +1] and
// 2 |J_perp| [coupled spin agrees with the sign of J_perp] are summed as 4 bytes at once without carries;
// per row only the field is added and the sum clamped to [-I_0, I_0 - 1] (Eq. 6b with alpha = 1).
// Otherwise each row's input is assembled in 32 bits and clamped as Eq. 6b states for any alpha.
template <bool kUpdate, bool kFast, int kMode, int kUnits, bool kFp4, bool kWide = false, class AccT>
__device__ __forceinline__ void fused_epilogue(const AccT& acc, v4i (&cnt)[kUnits][2], const EpilogueCtx& x) {
    // Per-lane addressing is rebuilt here from a laundered lane index, so that none of it stays live (in
    // registers) across the K loop.
    int ln = x.lane;
    asm volatile("" : "+v"(ln));
    auto ucol = [&](const int u) { return x.coff + (kWide ? 32 * (u >> 1) + (ln & 31) : 16 * u + (ln & 15)); };
    auto urun = [&](const int u) { return kWide ? 2 * (u & 1) + (ln >> 5) : (ln >> 4); };
    auto ucnt = [&](const int u) { return x.is_wg + (size_t)ucol(u) * x.np + x.tile * kTileRows + 32 * urun(u); };
    // clamp bounds of Eq. 6b, shifted by the accumulator's offset (its low byte is zero, so the low byte of a
    // shifted counter is the counter)
    constexpr int kOff = kFp4 ? 0x4B400000 : 0;
    const int lo = kOff - x.i0, hi = kOff + x.i0 - 1;
    const uint32_t tn2 = (uint32_t)x.two_n * 0x00010001u;
    const uint32_t tq2 = (uint32_t)x.two_q * 0x00010001u;

    // With 128-column blocks (one wave per SIMD, 512 registers) the LDS words the epilogue reads are read
    // ahead of the LDS writes that precede their use: the compiler cannot tell that those writes (the next
    // bit plane, the energy sums) leave them unchanged, so a read placed after a write is issued there and
    // waited for at once, with no other wave to absorb the latency.  The energy term's row constants of the
    // lane's runs are read once (8 x 16 bytes per run and lane; 32 x 32 tiles alternate between two runs), the
    // column table entries of all units next, and the bit-plane and noise words of unit u + 1 while unit u is
    // worked on.  Narrower blocks, whose two waves per SIMD cover each other's
    // latency, have no registers to spare for this and read each word where it is used.
    constexpr bool kAhead = kUnits == 8;
    v4i er[8], er1[8];
    uint32_t info_u[kUnits];
    auto read_er = [&](v4i (&dst)[8], const int u) {
#pragma unroll
        for (int ai = 0; ai < 8; ++ai) dst[ai] = *reinterpret_cast<const v4i*>(x.rows + 128 + 32 * urun(u) + 4 * ai);
    };
    if constexpr (kAhead) {
        read_er(er, 0);
        if constexpr (kWide) read_er(er1, 1);
#pragma unroll
        for (int u = 0; u < kUnits; ++u) info_u[u] = x.colinfo[ucol(u)];
    }
    uint32_t nx_sig = 0, nx_up = 0, nx_dn = 0, nx_noise = 0;
    auto read_words = [&](const int u) {
        const int c = ucol(u);
        const int word = x.tile * 4 + urun(u);
        if constexpr (!kAhead) info_u[u] = x.colinfo[c];
        nx_sig = ~x.pl_cur[c * x.cstride + word];
        if (kUpdate) {
            nx_up = x.pl_del[(info_u[u] & 0xFFu) * x.cstride_dn + word - x.dn_off];
            if (kMode == 1) nx_dn = x.pl_del[((info_u[u] >> 8) & 0xFFu) * x.cstride_dn + word - x.dn_off];
            nx_noise = x.noise_lds[(x.wave * x.ncols + c) * 4 + urun(u)];
        }
    };
    if constexpr (kAhead) read_words(0);

#pragma unroll
    for (int u = 0; u < kUnits; ++u) {
        const int c = ucol(u);
        const int word = x.tile * 4 + urun(u);
        if constexpr (!kAhead) read_words(u);
        const uint32_t info = info_u[u];
        const uint32_t nsig = nx_sig;
        uint32_t up_w = nx_up, dn_w = nx_dn, noise_w = nx_noise;
        if (kAhead && u + 1 < kUnits) read_words(u + 1);
        // four independent partial sums (one per byte position j), so that the energy is not one long chain
        int ep4[4] = {__builtin_popcount(nsig), 0, 0, 0};
        uint32_t negbits = 0;
        v4i* is_ptr = reinterpret_cast<v4i*>(ucnt(u));
        // With 32 x 32 tiles a unit's counters are half of a 128-byte line whose other half the next unit reads:
        // those go through the caches with either operand type, two units ahead.
        constexpr int kCnt = cnt_ahead<kFp4 || kWide>();
        if (kUpdate && u + kCnt < kUnits) load_counters_at<kFp4 || kWide>(cnt[u + kCnt], ucnt(u + kCnt));
        v4i is_lo = cnt[u][0], is_hi = cnt[u][1];
        if (kUpdate && kFast) {
            up_w ^= x.qflip;
            dn_w ^= x.qflip;
        }
#pragma unroll
        for (int ai = 0; ai < 8; ++ai) {
            const v4i er4 = kAhead ? ((kWide && (u & 1)) ? er1[ai] : er[ai])
                                   : *reinterpret_cast<const v4i*>(x.rows + 128 + 32 * urun(u) + 4 * ai);
            uint32_t isw_new = 0;
            int nvs[4] = {0, 0, 0, 0};
            const int isw = kUpdate ? (ai < 4 ? is_lo[ai] : is_hi[ai - 4]) : 0;
            uint32_t s4 = 0;
            if (kUpdate && kFast) {
                uint32_t c4 = (up_w >> ai) & 0x01010101u;
                if (kMode == 1) c4 += (dn_w >> ai) & 0x01010101u;
                const u16x2 t = __builtin_bit_cast(u16x2, nibble_to_bytes(noise_w, ai)) * __builtin_bit_cast(u16x2, tn2) +
                                __builtin_bit_cast(u16x2, c4) * __builtin_bit_cast(u16x2, tq2);
                s4 = (uint32_t)xad_u32(isw, (int)0x80808080u, (int)__builtin_bit_cast(uint32_t, t));
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int pos = 8 * j + ai;
                // the counter input without Is and the noise and coupling bytes (plus 0x4B400000 with fp4)
                const int f2 = acc_value<kUnits == 8>(acc, u, ai, j);
                // energy: (e ^ -1) = -e - 1 for sigma = -1; the -1s are restored by the popcount of nsig
                ep4[j] = xad_u32(f2 + er4[j], bfe_i((int)nsig, pos, 1), ep4[j]);
                if (kUpdate) {
                    const int base = f2;
                    int nv;
                    if (kFast) {
                        nv = med3_i32(base + (int)bfe_u(s4, 8 * j, 8), lo, hi);
                    } else {
                        int t = (bfe_i((int)noise_w, 4 * ai + j, 1) & x.two_n) + (bfe_i((int)up_w, pos, 1) & x.two_q);
                        if (kMode == 1) t += bfe_i((int)dn_w, pos, 1) & x.two_q;
                        const int sv = base + t + bfe_i(isw, 8 * j, 8);
                        nv = sv > hi ? x.i0 - x.alpha : (sv < lo ? lo : sv);
                    }
                    nvs[j] = nv;
                }
            }
            if (kUpdate) {
                // The low bytes of the four new counters into one dword, as a tree of byte permutes (selector byte
                // 0..3 picks a byte of the second operand, 4..7 of the first, 0x0C gives zero) rather than a chain
                // of four byte inserts, whose dependences a one-wave SIMD cannot hide.
                const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)nvs[1], (uint32_t)nvs[0], 0x0C0C0400u);
                const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)nvs[3], (uint32_t)nvs[2], 0x04000C0Cu);
                isw_new = p01 | p23;
                // sign bit of byte j (bit 8 j + 7) -> bit 8 j + a of the plane word
                negbits |= (isw_new >> (7 - ai)) & (0x01010101u << ai);
                if (ai < 4) is_lo[ai] = (int)isw_new; else is_hi[ai - 4] = (int)isw_new;
            }
        }
        if (kUpdate) {
            __builtin_nontemporal_store(is_lo, is_ptr);
            __builtin_nontemporal_store(is_hi, is_ptr + 1);
            x.pl_next[c * x.cstride_dn + word - x.dn_off] = ~negbits;
        }
        // Each lane adds its 32 rows' share: the lanes of a column meet in the LDS atomic, which needs no lane
        // index (a cross-lane shuffle would need one, and with every register taken the compiler reloads it
        // from scratch, whose wait then also drains the counter stores just issued).
        const int ep = (ep4[0] + ep4[1]) + (ep4[2] + ep4[3]);
        if (info >> 31) atomicAdd(&x.e_acc[c], ep);
    }
}

// Workgroup state shared by the sweep kernels: the sigma bit-plane ring and the per-column and per-trial
// accumulators in LDS (layout in sweep_block).
struct BlockLds {
    uint32_t* planes;     // [npl][kNB][cstride] sigma bit planes, npl = ring length (row-split: sigma(t) only)
    uint32_t* del_c;      // row-split form: [kNB][kGroupWords] the group's rows of sigma(t - d)
    uint32_t* next_c;     // row-split form: [kNB][kGroupWords] the group's rows of sigma(t + 1)
    int npl, plane_words, cstride;
    int32_t* e_acc;       // [kNB]
    int32_t* hit_l;       // [kNB]
    long long* best_l;    // [kNB]
    uint32_t* colinfo;    // [kNB]
};

// Column table, per-trial minima and first hits, and sigma(t_begin - s), s = 0..d, with the counters: drawn from
// the random stream (tag 0) at t_begin = 0, else taken from the counters and the saved history.
template <int kNB>
__device__ __forceinline__ void block_init(const SweepArgs& a, const int wg, const BlockLds& L) {
    uint32_t* planes = L.planes;
    const int npl = L.npl, plane_words = L.plane_words, cstride = L.cstride;
    int32_t* e_acc = L.e_acc;
    int32_t* hit_l = L.hit_l;
    long long* best_l = L.best_l;
    uint32_t* colinfo = L.colinfo;
    const int np = a.prob.np;
    const int tid = threadIdx.x;
    const int ntiles = np / kTileRows;
    const int R = a.R;
    const int b0 = wg * a.tpw;
    const int words = np / 32;
    int8_t* is_wg = a.is_state + (size_t)wg * kNB * np;

    for (int c = tid; c < kNB; c += kThreads) {
        e_acc[c] = 0;
        // column c = lb R + k: its ring neighbours k + 1 and k - 1 (mod R) and whether it is a real trial
        const int lb = c / R;
        const int k = c - lb * R;
        const bool real = c < a.cols_wg;
        const bool valid = real && (b0 + lb < a.T);
        const int c_up = real ? lb * R + (k + 1 == R ? 0 : k + 1) : c;
        const int c_dn = real ? lb * R + (k == 0 ? R - 1 : k - 1) : c;
        colinfo[c] = (uint32_t)c_up | ((uint32_t)c_dn << 8) | ((uint32_t)k << 16) | ((uint32_t)(lb & 0x7F) << 24) |
                     ((uint32_t)valid << 31);
    }
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
                const uint32_t sp = spread_bits(x.v[w]);
                for (int s = 0; s <= a.delay; ++s) {
                    const int p = (npl - s) % npl;
                    planes[p * plane_words + c * cstride + tile * 4 + w] = sp;
                }
                v4i* dst = reinterpret_cast<v4i*>(is_wg + (size_t)c * np + tile * kTileRows + 32 * w);
                v4i lo, hi;
                for (int q = 0; q < 4; ++q) {
                    uint32_t d0 = 0, d1 = 0;
                    for (int m = 0; m < 4; ++m) {
                        const uint32_t v0 = ((x.v[w] >> (4 * q + m)) & 1u) ? 0u : (uint32_t)(-a.alpha) & 0xFFu;
                        const uint32_t v1 = ((x.v[w] >> (16 + 4 * q + m)) & 1u) ? 0u : (uint32_t)(-a.alpha) & 0xFFu;
                        d0 |= v0 << (8 * m);
                        d1 |= v1 << (8 * m);
                    }
                    lo[q] = (int)d0;
                    hi[q] = (int)d1;
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
            for (int o = 0; o < 32; ++o) {
                const int word = (o < 16) ? lo[(o >> 2) & 3] : hi[(o >> 2) & 3];
                const int v = bfe_i(word, 8 * (o & 3), 8);
                bits |= (uint32_t)(v >= 0) << bitpos(o);
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
}

// End of cycle t: each replica's H_p (trace), the per-trial minimum and first hit; clears e_acc.  Wave w
// takes trials w, w + kWaves, ...: lane k reads replica k (and k + 64, ...), the minimum is reduced across
// the wave, and the lanes that read an entry clear it (entries of idle columns are never written).  H_p fits
// in 32 bits (|sum_i sigma_i (2 h_i + F_i)| < 2^30 by the problem's range check), so the minimum is taken in
// 32 bits with lane swizzles, which, unlike a shuffle, need no lane index in a register.
template <int kNB>
__device__ __forceinline__ void cycle_close(const SweepArgs& a, const int wg, const int t, const BlockLds& L) {
    int32_t* e_acc = L.e_acc;
    int32_t* hit_l = L.hit_l;
    long long* best_l = L.best_l;
    const int ln = __lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int R = a.R;
    const int b0 = wg * a.tpw;
    __syncthreads();

    // H_p of every replica at cycle t: sum_i sigma_i (2 h_i + F_i) = -2 H_p.
    for (int lb = wv; lb < a.tpw; lb += kWaves) {
        const int b = b0 + lb;
        int m = INT32_MAX;
        for (int k = ln; k < R; k += 64) {
            const int c = lb * R + k;
            const int e = -e_acc[c] / 2;
            if (b < a.T && a.trace) a.trace[(size_t)t * a.T * R + (size_t)b * R + k] = e;
            m = e < m ? e : m;
            e_acc[c] = 0;
        }
        // minimum over each 32-lane half (swizzle bitmask mode: lane j reads lane j ^ x), then over the halves
        int o = __builtin_amdgcn_ds_swizzle(m, (1 << 10) | 0x1F);
        m = o < m ? o : m;
        o = __builtin_amdgcn_ds_swizzle(m, (2 << 10) | 0x1F);
        m = o < m ? o : m;
        o = __builtin_amdgcn_ds_swizzle(m, (4 << 10) | 0x1F);
        m = o < m ? o : m;
        o = __builtin_amdgcn_ds_swizzle(m, (8 << 10) | 0x1F);
        m = o < m ? o : m;
        o = __builtin_amdgcn_ds_swizzle(m, (16 << 10) | 0x1F);
        m = o < m ? o : m;
        const int lo = __builtin_amdgcn_readlane(m, 0), hi = __builtin_amdgcn_readlane(m, 32);
        const long long mm = lo < hi ? lo : hi;
        if (ln == 0 && b < a.T) {
            if (mm < best_l[lb]) best_l[lb] = mm;
            if (hit_l[lb] < 0 && a.target != INT64_MIN && mm == a.target) hit_l[lb] = t;
        }
    }
    __syncthreads();
}

template <int kNB>
__device__ __forceinline__ void block_close(const SweepArgs& a, const int wg, const BlockLds& L) {
    const uint32_t* planes = L.planes;
    const int npl = L.npl, plane_words = L.plane_words, cstride = L.cstride;
    const int32_t* hit_l = L.hit_l;
    const long long* best_l = L.best_l;
    const int tid = threadIdx.x;
    const int b0 = wg * a.tpw;
    const int words = a.prob.np / 32;
    for (int lb = tid; lb < a.tpw; lb += kThreads) {
        const int b = b0 + lb;
        if (b < a.T) {
            a.best[b] = best_l[lb];
            a.first_hit[b] = hit_l[lb];
        }
    }
    if (a.save_hist && a.delay > 0) {
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

// ---------------------------------------------------------------------------------------------
// Row-split form: a trial's rows are spread over the row groups of its column block, one launch per cycle.
// ---------------------------------------------------------------------------------------------

// Row tiles [lo, hi) of row group g.
struct TileRange {
    int lo, hi;
};
__device__ __forceinline__ TileRange group_tiles(const SweepArgs& a, int g) {
    const int ntiles = a.prob.np / kTileRows;
    const int lo = min(g * a.group_tiles, ntiles);
    return TileRange{lo, min(lo + a.group_tiles, ntiles)};
}

// K steps [lo, hi) of wave `wave` when the four waves of a row-split workgroup share one tile: the ns steps
// (ns even) in pairs, as evenly as they go, wave 0 taking the last share (its range ends the product, so its
// counter prefetch in the last steps precedes the epilogue it runs).  Every share has at least two pairs when
// ns >= 16.
__device__ __forceinline__ TileRange k_share(int ns, int wave) {
    const int pairs = ns / 2, idx = kWaves - 1 - wave;
    const int base = pairs / kWaves, extra = pairs % kWaves;
    const int lo = 2 * (idx * base + min(idx, extra));
    return TileRange{lo, lo + 2 * (base + (idx < extra ? 1 : 0))};
}

// sigma(0) and Is(0) of group g's rows of column block cb from the random stream (tag 0), into the ring slots
// of sigma(0) and sigma(-s), s = 1..d; group 0 also resets the block's best energies, first hits and energy sums.
template <int kNB>
__device__ void split_init_state(const SweepArgs& a, const int cb, const int g) {
    const int np = a.prob.np, words = np / 32, npl = a.delay + 2;
    const int R = a.R, b0 = cb * a.tpw;
    const TileRange tr = group_tiles(a, g);
    int8_t* is_wg = a.is_state + (size_t)cb * kNB * np;
    for (int u = threadIdx.x; u < (tr.hi - tr.lo) * kNB; u += kThreads) {
        const int tile = tr.lo + u / kNB;
        const int c = u % kNB;
        const int k = c % R;
        const int b = b0 + c / R;
        const Philox4 x = philox4x32_10(0u, (uint32_t)tile, (uint32_t)k, (uint32_t)b, a.key0, a.key1);
        for (int w = 0; w < 4; ++w) {
            const uint32_t sp = spread_bits(x.v[w]);
            for (int s = 0; s <= a.delay; ++s) {
                const int p = (npl - s) % npl;
                a.ring[(((size_t)p * a.n_cb + cb) * kNB + c) * words + tile * 4 + w] = sp;
            }
            v4i* dst = reinterpret_cast<v4i*>(is_wg + (size_t)c * np + tile * kTileRows + 32 * w);
            v4i lo, hi;
            for (int q = 0; q < 4; ++q) {
                uint32_t d0 = 0, d1 = 0;
                for (int m = 0; m < 4; ++m) {
                    const uint32_t v0 = ((x.v[w] >> (4 * q + m)) & 1u) ? 0u : (uint32_t)(-a.alpha) & 0xFFu;
                    const uint32_t v1 = ((x.v[w] >> (16 + 4 * q + m)) & 1u) ? 0u : (uint32_t)(-a.alpha) & 0xFFu;
                    d0 |= v0 << (8 * m);
                    d1 |= v1 << (8 * m);
                }
                lo[q] = (int)d0;
                hi[q] = (int)d1;
            }
            dst[0] = lo;
            dst[1] = hi;
        }
    }
    if (g == 0) {
        for (int lb = threadIdx.x; lb < a.tpw; lb += kThreads) {
            const int b = b0 + lb;
            if (b < a.T) {
                a.best[b] = INT64_MAX;
                a.first_hit[b] = -1;
            }
        }
        // both energy-sum slots of the block start at zero (a kernel store, not a memset, so that a caller may
        // capture the launches in a graph)
        for (int c = threadIdx.x; c < kNB; c += kThreads) {
            a.e_sum[(size_t)cb * kNB + c] = 0;
            a.e_sum[(size_t)(a.n_cb + cb) * kNB + c] = 0;
        }
    }
}

// Cycle t of column block cb, once every row group has added its energy sums (the previous launch): each
// replica's H_p (trace), the per-trial minimum and first hit in device memory; the sums are cleared for cycle
// t + 2.  One wave, lane c on column c = lb R + k (trial lb, replica k; a block has at most 64 columns): every
// load is issued at once, and each trial's minimum is folded onto its replica-0 lane by a segmented reduction.
template <int kNB>
__device__ void split_close_cycle(const SweepArgs& a, const int cb, const int t) {
    static_assert(kNB <= 64, "the row-split form takes blocks of at most 64 columns");
    if (threadIdx.x >= 64) return;
    const int c = threadIdx.x;
    const int R = a.R;
    const int lb = c / R, k = c - lb * R;
    const int b = cb * a.tpw + lb;
    const bool real = c < a.cols_wg && b < a.T;
    const bool head = real && k == 0;
    int32_t* sums = a.e_sum + (size_t)(t & 1) * a.n_cb * kNB + (size_t)cb * kNB;
    const long long best = head ? a.best[b] : 0;
    const int hit = head ? a.first_hit[b] : 0;
    int m = INT32_MAX;
    if (c < kNB) {
        const int e = -sums[c] / 2;
        sums[c] = 0;
        if (real) {
            m = e;
            if (a.trace) a.trace[((size_t)t * a.T + b) * R + k] = e;
        }
    }
    // Lane c takes the minimum of lanes c .. c + 2 off - 1 of its trial; lanes past the trial's last replica
    // (k + off >= R) are never read, so the reads stay below lane a.cols_wg <= 64.
    for (int off = 1; off < R; off <<= 1) {
        const int o = __shfl_down(m, off, 64);
        if (k + off < R) m = o < m ? o : m;
    }
    if (head) {
        const long long mm = m;
        if (mm < best) a.best[b] = mm;
        if (hit < 0 && a.target != INT64_MIN && mm == a.target) a.first_hit[b] = t;
    }
}

// Workgroup state of one split launch at cycle a.t_begin: the column table, cleared energy sums, sigma(t) of
// every row and sigma(t - d) of the group's rows from the ring in device memory.
template <int kNB>
__device__ __forceinline__ void split_block_init(const SweepArgs& a, const int cb, const TileRange tr, const BlockLds& L) {
    const int np = a.prob.np, words = np / 32;
    const int npl = L.npl, cstride = L.cstride;
    const int R = a.R, b0 = cb * a.tpw;
    const int t = a.t_begin;
    const int tid = threadIdx.x;
    for (int c = tid; c < kNB; c += kThreads) {
        L.e_acc[c] = 0;
        const int lb = c / R;
        const int k = c - lb * R;
        const bool real = c < a.cols_wg;
        const bool valid = real && (b0 + lb < a.T);
        const int c_up = real ? lb * R + (k + 1 == R ? 0 : k + 1) : c;
        const int c_dn = real ? lb * R + (k == 0 ? R - 1 : k - 1) : c;
        L.colinfo[c] = (uint32_t)c_up | ((uint32_t)c_dn << 8) | ((uint32_t)k << 16) | ((uint32_t)(lb & 0x7F) << 24) |
                       ((uint32_t)valid << 31);
    }
    const int p_cur = t % npl;
    // sigma(t) of the whole block: 16-byte loads (a column's np / 32 words are a multiple of 4), four per
    // thread issued before any is stored, so that a block of up to 4096 rows arrives in one memory latency
    // instead of one per 256 words.
    const uint4* src = reinterpret_cast<const uint4*>(a.ring + ((size_t)p_cur * a.n_cb + cb) * kNB * words);
    const int n4 = kNB * words / 4;
    constexpr int kBatch = 4;
    for (int u0 = tid; u0 < n4; u0 += kBatch * kThreads) {
        uint4 v[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            if (u0 + i * kThreads < n4) v[i] = src[u0 + i * kThreads];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int u = u0 + i * kThreads;
            if (u < n4) {
                const int c = 4 * u / words;
                uint32_t* dst = L.planes + c * cstride + (4 * u - c * words);
                dst[0] = v[i].x;
                dst[1] = v[i].y;
                dst[2] = v[i].z;
                dst[3] = v[i].w;
            }
        }
    }
    {
        // the group's rows of sigma(t - d) (of sigma(t) when d = 0)
        const int p_del = (t - a.delay + npl) % npl;
        const uint32_t* dsrc = a.ring + ((size_t)p_del * a.n_cb + cb) * kNB * words;
        const int gw = 4 * (tr.hi - tr.lo);
        for (int u = tid; u < kNB * gw; u += kThreads) {
            const int c = u / gw;
            const int wl = u - c * gw;
            L.del_c[c * kGroupWords + wl] = dsrc[(size_t)c * words + 4 * tr.lo + wl];
        }
    }
    __syncthreads();
}

// End of a split launch: sigma(t + 1) of the group's rows back to the ring, and the group's energy sums added
// to the column block's totals for cycle t.
template <int kNB>
__device__ __forceinline__ void split_block_close(const SweepArgs& a, const int cb, const TileRange tr, const int t,
                                                  const bool update, const BlockLds& L) {
    const int np = a.prob.np, words = np / 32;
    __syncthreads();
    if (update) {
        const int p_next = (t + 1) % L.npl;
        uint32_t* dst = a.ring + ((size_t)p_next * a.n_cb + cb) * kNB * words;
        const int gw = 4 * (tr.hi - tr.lo);
        for (int u = threadIdx.x; u < kNB * gw; u += kThreads) {
            const int c = u / gw;
            const int wl = u - c * gw;
            dst[(size_t)c * words + 4 * tr.lo + wl] = L.next_c[c * kGroupWords + wl];
        }
    }
    if (tr.hi > tr.lo) {
        int32_t* sums = a.e_sum + (size_t)(t & 1) * a.n_cb * kNB + (size_t)cb * kNB;
        for (int c = threadIdx.x; c < kNB; c += kThreads)
            if (L.colinfo[c] >> 31) atomicAdd(&sums[c], L.e_acc[c]);
    }
}

// LDS layout of one workgroup (dynamic shared memory, 32-bit words):
//   planes  [d + 2][kNB][np / 32 + 1]   sigma bit planes (ring), kNB = 16 kNBF columns
//   noise   [kWaves][kNB][4]            one Philox block per column, exchanged inside the wave
//   e_acc   [kNB]   int32               sum_i sigma_i (2 h_i + F_i) per column, this cycle
//   hit     [kNB]   int32               per-trial first hit
//   best    [kNB]   int64               per-trial best energy
//   colinfo [kNB]   u32                 ring neighbours, replica and trial of each column
//   rows    [kWaves][256] int32         row vectors of each wave's current tile
// All cycles [a.t_begin, a.t_end] of column block `wg` of one anneal (a persistent workgroup).
// With kSplit, one cycle (a.t_begin) of row group `group` of column block `wg` (the row-split form).
template <bool kFast, int kMode, int kNBF, bool kFp4, bool kSplit = false>
__device__ __forceinline__ void sweep_block(const SweepArgs& a, const int wg, const int group = 0) {
    constexpr int kNB = 16 * kNBF;
    extern __shared__ uint32_t lds[];
    const int np = a.prob.np;
    const int cstride = plane_stride(np);
    const int plane_words = kNB * cstride;
    const int npl = a.delay + 2;
    uint32_t* planes = lds;
    // The row-split form holds sigma(t) of the whole block and only the group's rows of sigma(t - d) and
    // sigma(t + 1) (kGroupWords words per column), so that large N keep two workgroups per CU.
    uint32_t* del_c = lds + plane_words;
    uint32_t* next_c = del_c + kNB * kGroupWords;
    uint32_t* noise_lds = kSplit ? next_c + kNB * kGroupWords : lds + npl * plane_words;
    int32_t* e_acc = reinterpret_cast<int32_t*>(noise_lds + kWaves * kNB * 4);
    int32_t* hit_l = e_acc + kNB;
    long long* best_l = reinterpret_cast<long long*>(hit_l + kNB);
    uint32_t* colinfo = reinterpret_cast<uint32_t*>(best_l + kNB);   // [kNB]
    int32_t* rowst = reinterpret_cast<int32_t*>(colinfo + kNB);      // [kWaves][256]
    v4i* red = reinterpret_cast<v4i*>(rowst + kWaves * 256);          // [3 kNB / 2][64] v4i (split_k = 4)

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: keeps tile offsets scalar
    const int ntiles = np / kTileRows;
    const int nsteps = np / kStepK;
    const int b0 = wg * a.tpw;
    int8_t* is_wg = a.is_state + (size_t)wg * kNB * np;

    const BlockLds L{planes, kSplit ? del_c : nullptr, kSplit ? next_c : nullptr, npl, plane_words, cstride,
                     e_acc, hit_l, best_l, colinfo};
    // Row tiles of this workgroup: all of them, or the group's range in the row-split form.
    const TileRange tr = kSplit ? group_tiles(a, group) : TileRange{0, ntiles};
    // The row-split form fetches its first tile's row vectors ahead of the block state, so that they are on
    // their way while sigma arrives from device memory.
    v4i rowv_first{};
    if constexpr (kSplit) {
        const int ft = (kNBF == 2 && a.split_k == 4) ? tr.lo : tr.lo + wave;
        rowv_first = fetch_rows(a.prob, ft < tr.hi ? ft : ntiles - 1);
    }
    if constexpr (kSplit) split_block_init<kNB>(a, wg, tr, L);
    else block_init<kNB>(a, wg, L);

    // 128-column blocks with int8 operands take single-plane problems only (the host checks it): a Horner
    // update of 256 AGPR accumulators would need more VGPRs than are left beside them.
    const int P = (kNBF == 8 && !kFp4) ? 1 : a.prob.planes;
    // Buffer resource over all J planes (gfx9 raw buffer, byte addressed).
    const __amdgpu_buffer_rsrc_t jrsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t*>(a.prob.J), 0, P * np * np, 0x00020000);
    const __amdgpu_buffer_rsrc_t j4rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(a.prob.J4), 0, kFp4 ? np * (a.prob.kp4 / 2) : 0, 0x00020000);

    // The row-split form runs one cycle (t_begin) per launch: its loop has one trip, which the compiler then
    // lays out straight instead of hoisting the cycle's set-up into a preheader.
    const int t_last = kSplit ? a.t_begin : a.t_end;
    for (int t = a.t_begin; t <= t_last; ++t) {
        const bool update = t < a.t_end;
        if (!update && !a.final_pass) break;
        const int p_cur = t % npl;
        const int p_next = (t + 1) % npl;
        const int p_del = (t - a.delay + npl) % npl;
        const int q = update ? (kSplit ? a.split_q : a.jperp[t]) : 0;
        const int i0 = update ? (kSplit ? a.split_i0 : a.i0[t]) : 0;
        // Counter input (Eq. 6a, with sigma = 2 x - 1 and F = 2 sum_j J_ij x_j - rowsum):
        //   s = Is + 2 sum_j J_ij x_j + (h - rowsum) - n_rnd - q (1 + mode) + 2 n_rnd [r = +1]
        //       + 2 q [sigma_up = +1] (+ 2 q [sigma_dn = +1] in mode 1).
        // The fast path writes q (2 [sigma = +1] - 1) as 2 |q| [sigma = sign q] - |q|.
        // The accumulator starts from the per-row part of s and collects 2 sum_j J_ij x_j, so that it ends as
        // v = s - Is - (the noise and coupling increments).  With fp4 operands it is an fp32 number 1.5 * 2^23 + v
        // with v an integer below 2^22 in magnitude, whose bits are kAccOffset + v; the epilogue works on those
        // bits directly.  With int8 operands it is v itself (int32).
        constexpr int kAccOffset = kFp4 ? 0x4B400000 : 0;
        const int qa = kFast ? (q < 0 ? -q : q) : q;
        const int two_n = 2 * a.noise_amp;
        const int two_q = 2 * qa;
        const int adj = -a.noise_amp - qa * (kMode == 1 ? 2 : 1);
        // The fast path adds the counters offset by 128, which the per-row constant takes back.
        const int adj_c = adj - (kFast ? 128 : 0);
        // Per-row constants staged with each tile (see the tile loop): the first vector (h - rowsum) gets
        // row_add_h, the second (h) gets row_add_e.
        const int row_add_h = adj_c + kAccOffset;
        const int row_add_e = -adj_c - kAccOffset;
        const uint32_t qflip = (kFast && q < 0) ? 0xFFFFFFFFu : 0u;
        const uint32_t* pl_cur = kSplit ? planes : planes + p_cur * plane_words;
        const uint32_t* pl_del = kSplit ? del_c : planes + p_del * plane_words;
        uint32_t* pl_next = kSplit ? next_c : planes + p_next * plane_words;

        // The work of one tile for kF column fragments starting at fragment foff: all of them (kF = kNBF,
        // foff = 0), or one column half of a 128-column block (kF = 4, foff = 0 or 4).
        v4i rowv_next;
        auto tile_body = [&](auto kF_c, const int tile, const int foff, const bool more, const int next_tile) {
            constexpr int kF = decltype(kF_c)::value;
            // Per-row constants of this tile, staged in LDS for the first K step and the epilogue: [0, 128) the
            // accumulator's start, kAccOffset + h - rowsum + adj_c (fp32 bits with fp4 operands), [128, 256)
            // h - adj_c - kAccOffset, so that start + 2 sum_j J_ij x_j + this = 2 h + F (the energy term).
            stage_rows(rowst + wave * 256, rowv_next, row_add_h, row_add_e);
            const int32_t* rows_w = rowst + wave * 256;
            // 128- and 64-column blocks with fp4 operands take 32 x 32 x 64 MFMAs (kWideT); 32-column fp4 blocks and
            // int8 operands on 64 and 32 columns take 16 x 16 ones.
            constexpr bool kWideT = kFp4 && (kNBF == 8 || kNBF == 4);
            // 128-column blocks with int8 operands (single-plane J) take int8 32 x 32 x 32 MFMAs (kWideI), in the
            // same output layout.
            constexpr bool kWideI = !kFp4 && kNBF == 8;
            constexpr int kNCB = kF / 2;
            v4i acc[8][kF];
            v16i accw[4][kNCB];
            // This lane's counters of the tile, fetched during the last K steps for the epilogue.
            v4i cnt[kF][2];
            // Lane-derived addresses are rebuilt per tile from a laundered lane index: held across the
            // epilogue they would be spilled, and reloading them in front of the K loop forces a wait for all
            // J loads in flight at the head of every K step.
            int tl = lane;
            asm volatile("" : "+v"(tl));
            const int tcol = tl & 15;
            const int tg = tl >> 4;
            int8_t* is_lane = is_wg + (size_t)(tcol + 16 * foff) * np + tile * kTileRows + 32 * tg;
            const int voff = tl * 16;
            // A row-split group of one tile with split_k = 4 (32-column blocks, which have the registers to spare):
            // the four waves share its K steps (k_share); wave 0 starts from the staged constants, and waves 0
            // and 1 each add the others' partial sums of one column fragment and run its epilogue.
            const bool share = kSplit && kNBF == 2 && a.split_k == 4;
            const bool lead = !share || wave == 0;
            // The epilogue's counters, fetched during the last K steps: every fragment's, or with `share` the
            // wave's own fragment's (waves 0 and 1) into slot 0.
            auto prefetch_epi = [&]() {
                if (!share) prefetch_counters<kF, kFp4>(cnt, is_lane, np);
                else if (wave < kF) load_counters<kFp4>(cnt[0], is_lane, np, wave);
            };
            if constexpr (kWideT) {
                // Field product on the fp4 copy of J (the same layout and exactness argument as below) with
                // 32 x 32 x 64 MFMAs: per K step of 128, row blocks rb < 4 of 32 rows, column blocks cb < kNCB
                // of 32 columns and K halves kh < 2.  Lane l loads the 16 bytes of J for operand row p = l % 32
                // and K half-group l / 32: row p of block rb is the layout's slot p % 16 of fragment
                // 2 rb + p / 16, so that each load reads two contiguous 512-byte runs, and output register
                // 4 i + j of the lane lands on tile row 64 (i & 1) + 32 (l / 32) + 8 rb + 4 (i >> 1) + j: two
                // runs of 32 consecutive rows per lane and column, as the epilogue's units want them.
                v16f accf[4][kNCB];
                const int ns = a.prob.kp4 / 128;          // even, >= 4
                const TileRange kr = share ? k_share(ns, wave) : TileRange{0, ns};
                const int jv = ((tl & 31) >> 4) * 1024 + ((tl >> 5) * 16 + (tl & 15)) * 16;
                const int tile_off = tile * ns * 8 * 1024;
                // Word 4 s + 2 kh + l / 32 of the lane's column for K step s (past the column's slot for the
                // last steps when kp4 > np, as below: J is zero there).
                const uint32_t* bsrc = pl_cur + (16 * foff + (tl & 31)) * cstride + (tl >> 5);
                v4i A0[2][4], A1[2][4];
                uint32_t w[2][kNCB], wn[2][kNCB];
                auto read_words = [&](uint32_t (&dst)[2][kNCB], int s) {
#pragma unroll
                    for (int kh = 0; kh < 2; ++kh)
#pragma unroll
                        for (int cb = 0; cb < kNCB; ++cb) dst[kh][cb] = bsrc[32 * cb * cstride + 4 * s + 2 * kh];
                };
                auto load_step = [&](v4i (&A)[2][4], int off) {
#pragma unroll
                    for (int kh = 0; kh < 2; ++kh)
#pragma unroll
                        for (int rb = 0; rb < 4; ++rb) A[kh][rb] = load_j(j4rsrc, jv, off + rb * 2048 + kh * 512);
                };
                load_step(A0, tile_off + kr.lo * 8 * 1024);
                load_step(A1, tile_off + (kr.lo + 1) * 8 * 1024);
                read_words(w, kr.lo);
                // The accumulators' starts (register 4 i + j of row block rb: the staged constant of its tile
                // row), read while the first J fragments are on their way.
                v16f start[4];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    v4i q[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        q[i] = *reinterpret_cast<const v4i*>(rows_w + 64 * (i & 1) + 32 * (tl >> 5) + 8 * rb + 4 * (i >> 1));
                    start[rb] = __builtin_bit_cast(v16f, (v16i){q[0][0], q[0][1], q[0][2], q[0][3], q[1][0], q[1][1], q[1][2],
                                                               q[1][3], q[2][0], q[2][1], q[2][2], q[2][3], q[3][0], q[3][1],
                                                               q[3][2], q[3][3]});
                    if (!lead) start[rb] = v16f{};
                }
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), as below
                v4i Bc = expand_operand_fp4(w[0][0]);
                read_words(wn, kr.lo + 1);
                mma_fp4_wide<kNCB, true, true, true>(A0, Bc, w, wn[0][0], accf, start, j4rsrc, jv,
                                                     tile_off + (kr.lo + 2) * 8 * 1024);
                read_words(w, kr.lo + 2);
                mma_fp4_wide<kNCB, true, true, false>(A1, Bc, wn, w[0][0], accf, start, j4rsrc, jv,
                                                      tile_off + (kr.lo + 3) * 8 * 1024);
                for (int s = kr.lo + 2; s < kr.hi - 2; s += 2) {
                    read_words(wn, s + 1);
                    mma_fp4_wide<kNCB, true, true, false>(A0, Bc, w, wn[0][0], accf, start, j4rsrc, jv,
                                                          tile_off + (s + 2) * 8 * 1024);
                    read_words(w, s + 2);
                    mma_fp4_wide<kNCB, true, true, false>(A1, Bc, wn, w[0][0], accf, start, j4rsrc, jv,
                                                          tile_off + (s + 3) * 8 * 1024);
                }
                read_words(wn, kr.hi - 1);
                mma_fp4_wide<kNCB, false, true, false>(A0, Bc, w, wn[0][0], accf, start, j4rsrc, jv, 0);
                if (more) rowv_next = fetch_rows(a.prob, next_tile);
                // the counters of the epilogue's first units (unit u: column 32 (u / 2) + l % 32, run 2 (u % 2) + l / 32)
                if (lead) {
                    const int8_t* p0 = is_wg + (size_t)(16 * foff + (tl & 31)) * np + tile * kTileRows + 32 * (tl >> 5);
#pragma unroll
                    for (int u = 0; u < kF && u < cnt_ahead<true>(); ++u)
                        load_counters_at<true>(cnt[u], p0 + (size_t)32 * (u >> 1) * np + 64 * (u & 1));
                }
                mma_fp4_wide<kNCB, false, false, false>(A1, Bc, wn, 0u, accf, start, j4rsrc, jv, 0);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < kNCB; ++cb) accw[rb][cb] = __builtin_bit_cast(v16i, accf[rb][cb]);
            } else if constexpr (kFp4) {
                // Field product on the fp4 copy of J: K steps of 128 with J scaled by 2, fp32 accumulators that
                // start from the staged per-row constant (1.5 * 2^23 plus an integer).  Every partial sum is
                // 1.5 * 2^23 plus an integer of magnitude below 2^22, so it is exact in any summation order and
                // its bits are 0x4B400000 plus that integer.
                v4f accf[8][kF];
                const int ns = a.prob.kp4 / 128;          // even, >= 4
                const TileRange kr = share ? k_share(ns, wave) : TileRange{0, ns};
                // Word 4 s + g of the lane's column for K step s.  When kp4 > np the last steps read up to
                // (kp4 - np) / 32 - 1 words past the column's slot (into the next column, or past the last
                // plane into the noise area): J is zero for those K, so the bits read there do not matter.
                const uint32_t* bsrc = pl_cur + (tcol + 16 * foff) * cstride + tg;
                const int tile_off = tile * ns * 8 * 1024;
                v4i A0[8], A1[8];
                // Bit-plane words of two consecutive K steps, used alternately (w: even steps, wn: odd steps).
                uint32_t w[kF], wn[kF];
                auto read_words = [&](uint32_t (&dst)[kF], int s) {
#pragma unroll
                    for (int f = 0; f < kF; ++f) dst[f] = bsrc[16 * f * cstride + 4 * s];
                };
                load_fragments(A0, j4rsrc, voff, tile_off + kr.lo * 8 * 1024);
                load_fragments(A1, j4rsrc, voff, tile_off + (kr.lo + 1) * 8 * 1024);
                read_words(w, kr.lo);
                // With 128-column blocks (512 registers) the staged accumulator starts of all eight row blocks are
                // read here, while the first J fragments are on their way: read one row block at a time in the
                // first K step, each read waits out the LDS latency on its own, with no other wave on the SIMD.
                // Narrower blocks have no registers to spare for them and read each where it is used.
                v4i start4[8];
                if constexpr (kNBF == 8) {
#pragma unroll
                    for (int ai = 0; ai < 8; ++ai) start4[ai] = *reinterpret_cast<const v4i*>(rows_w + 32 * tg + 4 * ai);
                }
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), as in the int8 loop
                // ns >= 4.  The J loads in flight at the head of the steady loop are the same, in the same order, on
                // entry and around the loop (A0 of step s + 2, then A1 of step s + 3), and every path into the loop
                // issues the same loads: otherwise the compiler waits for every load in flight at the head of each
                // iteration and the prefetch is lost.
                v4i Bc;
                {
                    // Step 0 starts every accumulator of row block ai from the staged constants.
                    v4i B[kF];
#pragma unroll
                    for (int f = 0; f < kF; ++f) B[f] = expand_operand_fp4(w[f]);
                    read_words(wn, kr.lo + 1);
#pragma unroll
                    for (int ai = 0; ai < 8; ++ai) {
                        v4f start = __builtin_bit_cast(
                            v4f, kNBF == 8 ? start4[ai] : *reinterpret_cast<const v4i*>(rows_w + 32 * tg + 4 * ai));
                        if (!lead) start = v4f{};
#pragma unroll
                        for (int f = 0; f < kF; ++f) accf[ai][f] = mfma_fp4(A0[ai], B[f], start);
                        A0[ai] = load_j(j4rsrc, voff, tile_off + (kr.lo + 2) * 8 * 1024 + ai * 1024);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    Bc = expand_operand_fp4(wn[0]);
                }
                read_words(w, kr.lo + 2);
                mma_fp4_cols<kF, true, true>(A1, Bc, wn, w[0], accf, j4rsrc, voff, tile_off + (kr.lo + 3) * 8 * 1024);
                // Steady state: each step reloads the A buffer it consumed with the fragments two steps ahead.
                for (int s = kr.lo + 2; s < kr.hi - 2; s += 2) {
                    read_words(wn, s + 1);
                    mma_fp4_cols<kF, true, true>(A0, Bc, w, wn[0], accf, j4rsrc, voff, tile_off + (s + 2) * 8 * 1024);
                    read_words(w, s + 2);
                    mma_fp4_cols<kF, true, true>(A1, Bc, wn, w[0], accf, j4rsrc, voff, tile_off + (s + 3) * 8 * 1024);
                }
                // The last two steps: no J left to fetch; the next tile's row vectors and the epilogue's counters
                // are fetched instead.
                read_words(wn, kr.hi - 1);
                mma_fp4_cols<kF, false, true>(A0, Bc, w, wn[0], accf, j4rsrc, voff, 0);
                if (more) rowv_next = fetch_rows(a.prob, next_tile);
                prefetch_epi();
                mma_fp4_cols<kF, false, false>(A1, Bc, wn, 0u, accf, j4rsrc, voff, 0);
#pragma unroll
                for (int ai = 0; ai < 8; ++ai)
#pragma unroll
                    for (int f = 0; f < kF; ++f) acc[ai][f] = __builtin_bit_cast(v4i, accf[ai][f]);
            } else if constexpr (kWideI) {
                // Field product on int8 J (one plane) with 32 x 32 x 32 MFMAs: per K step of 64, row blocks rb < 4,
                // column blocks cb < kNCB and K halves kh < 2 of 32.  Lane l loads the 16 bytes of J for operand row
                // p = l % 32 and K group 2 kh + l / 32 (slot p % 16 of fragment 2 rb + p / 16 of the int8 layout, as
                // on the fp4 path), and the operand 2 x of its 16 K values from half l / 32 of bit-plane word 2 s + kh.
                // The accumulators start from the staged constants (register 4 i + j of row block rb: tile row
                // 64 (i & 1) + 32 (l / 32) + 8 rb + 4 (i >> 1) + j) and end as the counter input v.
                const int jv = ((tl & 31) >> 4) * 1024 + ((tl >> 5) * 16 + (tl & 15)) * 16;
                const int tile_off = tile * nsteps * 8 * 1024;
                const uint32_t* bsrc = pl_cur + (16 * foff + (tl & 31)) * cstride;
                const int bsh = 4 * (tl >> 5);
                v4i A0[2][4], A1[2][4];
                uint32_t w[2][kNCB], wn[2][kNCB];
                auto read_words = [&](uint32_t (&dst)[2][kNCB], int s) {
#pragma unroll
                    for (int kh = 0; kh < 2; ++kh)
#pragma unroll
                        for (int cb = 0; cb < kNCB; ++cb) dst[kh][cb] = bsrc[32 * cb * cstride + 2 * s + kh];
                };
                auto load_step = [&](v4i (&A)[2][4], int off) {
#pragma unroll
                    for (int kh = 0; kh < 2; ++kh)
#pragma unroll
                        for (int rb = 0; rb < 4; ++rb) A[kh][rb] = load_j(jrsrc, jv, off + rb * 2048 + kh * 512);
                };
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    v4i q[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        q[i] = *reinterpret_cast<const v4i*>(rows_w + 64 * (i & 1) + 32 * (tl >> 5) + 8 * rb + 4 * (i >> 1));
                    const v16i st = (v16i){q[0][0], q[0][1], q[0][2], q[0][3], q[1][0], q[1][1], q[1][2], q[1][3],
                                           q[2][0], q[2][1], q[2][2], q[2][3], q[3][0], q[3][1], q[3][2], q[3][3]};
#pragma unroll
                    for (int cb = 0; cb < kNCB; ++cb) accw[rb][cb] = st;
                }
                load_step(A0, tile_off);
                load_step(A1, tile_off + 8 * 1024);
                read_words(w, 0);
                // Drain the first loads here, as below.
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
                v4i Bc = expand_operand(w[0][0] >> bsh);
                for (int s = 0; s < nsteps - 2; s += 2) {
                    read_words(wn, s + 1);
                    mma_i8_wide<kNCB, true, true>(A0, Bc, w, wn[0][0], bsh, accw, jrsrc, jv, tile_off + (s + 2) * 8 * 1024);
                    read_words(w, s + 2);
                    mma_i8_wide<kNCB, true, true>(A1, Bc, wn, w[0][0], bsh, accw, jrsrc, jv, tile_off + (s + 3) * 8 * 1024);
                }
                read_words(wn, nsteps - 1);
                mma_i8_wide<kNCB, false, true>(A0, Bc, w, wn[0][0], bsh, accw, jrsrc, jv, 0);
                if (more) rowv_next = fetch_rows(a.prob, next_tile);
                {
                    const int8_t* p0 = is_wg + (size_t)(16 * foff + (tl & 31)) * np + tile * kTileRows + 32 * (tl >> 5);
#pragma unroll
                    for (int u = 0; u < kF && u < cnt_ahead<true>(); ++u)
                        load_counters_at<true>(cnt[u], p0 + (size_t)32 * (u >> 1) * np + 64 * (u & 1));
                }
                mma_i8_wide<kNCB, false, false>(A1, Bc, wn, 0u, bsh, accw, jrsrc, jv, 0);
            } else {
                // Output slot (ai, r = col16) of every fragment is tile row 32 (r / 4) + 4 ai + r % 4, so lane
                // group g ends up with rows 32 g .. 32 g + 31.  The operand is 2 x, so the accumulators collect
                // 2 sum_j J_ij x_j on top of the staged start (the counter input v, as with fp4 operands).
                const uint32_t* bsrc = pl_cur + (tcol + 16 * foff) * cstride + (tg >> 1);
                const int bsh = 4 * (tg & 1);
                // Bit-plane words of two consecutive K steps, used alternately (w: even steps, wn: odd steps).
                uint32_t w[kF], wn[kF];
                auto read_words = [&](uint32_t (&dst)[kF], int s) {
#pragma unroll
                    for (int f = 0; f < kF; ++f) dst[f] = bsrc[16 * f * cstride + 2 * s];
                };
                // The accumulators start from the staged constants (for a single plane; zero when several planes
                // follow), and each later pass scales the running sum by 256 (exact Horner evaluation over the
                // planes), the last one adding the start.  Setting them takes the moves a zero start took before.
                const TileRange kr = share ? k_share(nsteps, wave) : TileRange{0, nsteps};
#pragma unroll
                for (int ai = 0; ai < 8; ++ai) {
                    v4i st = *reinterpret_cast<const v4i*>(rows_w + 32 * tg + 4 * ai);
                    if (P != 1 || !lead) st = v4i{0, 0, 0, 0};
#pragma unroll
                    for (int f = 0; f < kF; ++f) acc[ai][f] = st;
                }
                for (int p = P - 1; p >= 0; --p) {
                    if (p < P - 1) {   // never with 128 columns (P = 1 there)
#pragma unroll
                        for (int ai = 0; ai < 8; ++ai) {
                            v4i st = *reinterpret_cast<const v4i*>(rows_w + 32 * tg + 4 * ai);
                            if (p != 0 || !lead) st = v4i{0, 0, 0, 0};
#pragma unroll
                            for (int f = 0; f < kF; ++f) acc[ai][f] = acc[ai][f] * 256 + st;
                        }
                    }
                    // J is read through a buffer resource (loads past the planes return 0 instead of faulting),
                    // one contiguous 1 KiB fragment per load, into two A buffers: buffer b holds step s while the
                    // loads of step s + 2 refill it right behind the MFMAs that read it.
                    const int tile_off = p * np * np + tile * nsteps * 8 * 1024;
                    v4i A0[8], A1[8];
                    load_fragments(A0, jrsrc, voff, tile_off + kr.lo * 8 * 1024);
                    load_fragments(A1, jrsrc, voff, tile_off + (kr.lo + 1) * 8 * 1024);
                    read_words(w, kr.lo);
                    // Drain the first loads here: at the loop head the loads in flight are then exactly the ones
                    // the previous steps issued in fragment order, so each MFMA group waits for its own fragment.
                    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
                    v4i Bc = expand_operand(w[0] >> bsh);
                    int s = kr.lo;
                    for (; s < kr.hi - 2; s += 2) {
                        read_words(wn, s + 1);
                        mma_i8_cols<kF, true, true>(A0, Bc, w, wn[0], bsh, acc, jrsrc, voff, tile_off + (s + 2) * 8 * 1024);
                        read_words(w, s + 2);
                        mma_i8_cols<kF, true, true>(A1, Bc, wn, w[0], bsh, acc, jrsrc, voff, tile_off + (s + 3) * 8 * 1024);
                    }
                    // the last two steps: no J left to fetch
                    read_words(wn, kr.hi - 1);
                    mma_i8_cols<kF, false, true>(A0, Bc, w, wn[0], bsh, acc, jrsrc, voff, 0);
                    if (p == 0) {
                        if (more) rowv_next = fetch_rows(a.prob, next_tile);
                        prefetch_epi();
                    }
                    mma_i8_cols<kF, false, false>(A1, Bc, wn, 0u, bsh, acc, jrsrc, voff, 0);
                }
            }

            // ---------------- fused epilogue ----------------
            EpilogueCtx ctx;
            ctx.pl_cur = pl_cur;
            ctx.pl_del = pl_del;
            ctx.pl_next = pl_next;
            ctx.noise_lds = noise_lds;
            ctx.colinfo = colinfo;
            ctx.e_acc = e_acc;
            ctx.is_wg = is_wg;
            ctx.rows = rows_w;
            ctx.np = np;
            ctx.cstride = cstride;
            ctx.cstride_dn = kSplit ? kGroupWords : cstride;
            ctx.dn_off = kSplit ? 4 * tr.lo : 0;
            ctx.tile = tile;
            ctx.wave = wave;
            ctx.lane = lane;
            ctx.qflip = qflip;
            ctx.two_n = two_n;
            ctx.two_q = two_q;
            ctx.i0 = i0;
            ctx.alpha = a.alpha;
            ctx.coff = 16 * foff;
            ctx.ncols = kNB;
            // The column fragments this wave finishes: [ef, ef + efn).
            int ef = foff, efn = kF;
            v4i acc1[8][1];       // with `share`: the summed accumulators of fragment `wave`
            if constexpr (kSplit && kNBF == 2) {
                if (share) {
                    // Waves 2 and 3 pass all their partial sums through LDS, waves 0 and 1 the fragment the other
                    // one finishes; each of waves 0 and 1 then adds the three partial sums of its fragment to its
                    // own.  They are integers (with fp4 operands fp32 values below 2^22 in magnitude, as every
                    // partial sum of a row's product is), so the sum is exact in any order.
                    static_assert(kF == 2 && !(kWideT || kWideI), "shared tiles take 16 x 16 tiles of 32 columns");
                    constexpr int kV = 8 * kF;   // 16-byte vectors of accumulators per lane
                    auto slot = [&](const int i) -> v4i& { return red[(size_t)i * 64 + lane]; };
                    if (wave >= kF) {
#pragma unroll
                        for (int q = 0; q < kV; ++q) slot((wave - kF) * kV + q) = acc[q / kF][q % kF];
                    } else {
#pragma unroll
                        for (int ai = 0; ai < 8; ++ai) slot(2 * kV + 8 * wave + ai) = wave == 0 ? acc[ai][1] : acc[ai][0];
                    }
                    __syncthreads();
                    if (wave >= kF) return;
#pragma unroll
                    for (int ai = 0; ai < 8; ++ai) {
                        const v4i own = wave == 0 ? acc[ai][0] : acc[ai][1];
                        const v4i o2 = slot(ai * kF + wave), o3 = slot(kV + ai * kF + wave);
                        const v4i o1 = slot(2 * kV + 8 * (1 - wave) + ai);
                        if constexpr (kFp4)
                            acc1[ai][0] = __builtin_bit_cast(
                                v4i, (__builtin_bit_cast(v4f, own) + __builtin_bit_cast(v4f, o1)) +
                                         (__builtin_bit_cast(v4f, o2) + __builtin_bit_cast(v4f, o3)));
                        else
                            acc1[ai][0] = (own + o1) + (o2 + o3);
                    }
                    ef = wave;
                    efn = 1;
                    ctx.coff = 16 * wave;
                }
            }
            if (update) {
                // One Philox block per column (lane c computes columns c, c + 64, ...), shared through LDS
                // within the wave.
                for (int c = 16 * ef + lane; c < 16 * (ef + efn); c += 64) {
                    const uint32_t mine = colinfo[c];
                    const Philox4 x = philox4x32_10((uint32_t)(t + 1), (uint32_t)tile, (mine >> 16) & 0xFFu,
                                                    (uint32_t)b0 + ((mine >> 24) & 0x7Fu), a.key0, a.key1);
                    *reinterpret_cast<uint4*>(noise_lds + (wave * kNB + c) * 4) = uint4{x.v[0], x.v[1], x.v[2], x.v[3]};
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if constexpr (kSplit && kNBF == 2) {
                    if (share) {
                        v4i cnt1[1][2] = {{cnt[0][0], cnt[0][1]}};
                        fused_epilogue<true, kFast, kMode, 1, kFp4>(acc1, cnt1, ctx);
                        return;
                    }
                }
                if constexpr (kWideT || kWideI) fused_epilogue<true, kFast, kMode, kF, kFp4, true>(accw, cnt, ctx);
                else fused_epilogue<true, kFast, kMode, kF, kFp4>(acc, cnt, ctx);
            } else {
                if constexpr (kSplit && kNBF == 2) {
                    if (share) {
                        v4i cnt1[1][2] = {{cnt[0][0], cnt[0][1]}};
                        fused_epilogue<false, kFast, kMode, 1, kFp4>(acc1, cnt1, ctx);
                        return;
                    }
                }
                if constexpr (kWideT || kWideI) fused_epilogue<false, kFast, kMode, kF, kFp4, true>(accw, cnt, ctx);
                else fused_epilogue<false, kFast, kMode, kF, kFp4>(acc, cnt, ctx);
            }
        };
        // Tiles go to the waves in turn.  When whole rounds of the four waves leave one or two tiles over, those
        // are split into column halves (all 128 rows each), one per wave, so that the last round is shared instead
        // of leaving two or three waves idle.  64-column int8 blocks (whose half tiles would spill) and the
        // row-split form keep the plain loop.
        constexpr bool kCanSplit = kNBF == 8 || (kNBF == 4 && kFp4 && !kSplit) || (kNBF == 2 && !kSplit);
        if constexpr (kCanSplit) {
            const int rounds = ntiles / kWaves, left = ntiles % kWaves;
            const bool split = left == 1 || left == 2;
            const int n_full = split ? rounds : (ntiles - wave + kWaves - 1) / kWaves;
            const bool has_half = split && wave < 2 * left;
            const int half_tile = rounds * kWaves + (wave >> 1);
            // Row vectors of the wave's first tile; later tiles' are fetched during the previous tile's last K
            // steps.  A wave without work fetches the last tile's instead, so that the load stays inside the row
            // vectors.
            rowv_next = fetch_rows(a.prob, n_full > 0 ? wave : has_half ? half_tile : ntiles - 1);
            for (int i = 0; i < n_full; ++i) {
                const int tile = wave + kWaves * i;
                const bool last_full = i + 1 == n_full;
                tile_body(std::integral_constant<int, kNBF>{}, tile, 0, !last_full || has_half,
                          last_full ? half_tile : tile + kWaves);
            }
            if (has_half) tile_body(std::integral_constant<int, kNBF / 2>{}, half_tile, (wave & 1) * (kNBF / 2), false, 0);
        } else if (kSplit && kNBF == 2 && a.split_k == 4) {
            // a row group of one tile, whose K steps the four waves share
            rowv_next = rowv_first;
            if (tr.lo < tr.hi) tile_body(std::integral_constant<int, kNBF>{}, tr.lo, 0, false, 0);
        } else {
            // A wave without a tile (fewer tiles than waves) fetches the last tile's row vectors instead, so that
            // the load stays inside the row vectors; it never uses them.
            rowv_next = kSplit ? rowv_first : fetch_rows(a.prob, tr.lo + wave < tr.hi ? tr.lo + wave : ntiles - 1);
            for (int tile = tr.lo + wave; tile < tr.hi; tile += kWaves)
                tile_body(std::integral_constant<int, kNBF>{}, tile, 0, tile + kWaves < tr.hi, tile + kWaves);
        }
        if constexpr (kSplit) split_block_close<kNB>(a, wg, tr, t, update, L);
        else cycle_close<kNB>(a, wg, t, L);
    }

    if constexpr (!kSplit) block_close<kNB>(a, wg, L);
}

template <bool kFast, int kMode, int kNBF, bool kFp4>
__global__ __launch_bounds__(kThreads, kNBF == 8 ? 1 : 2) void sweep_kernel(SweepArgs a) {
    sweep_block<kFast, kMode, kNBF, kFp4>(a, blockIdx.x);
}

// One cycle t of a row-split anneal (flags kSplit*): workgroup blockIdx.x is row group blockIdx.x % n_groups of
// column block blockIdx.x / n_groups, so that with n_groups a multiple of the XCD count every column block's
// copy of a row group runs on one XCD and their J rows meet in its L2.
template <bool kFast, int kMode, int kNBF, bool kFp4>
__global__ __launch_bounds__(kThreads, 2) void sweep_split_kernel(const SweepArgs* __restrict__ item, int t, int flags,
                                                                   int q_t, int i0_t) {
    SweepArgs a = *item;
    const int cb = blockIdx.x / a.n_groups;
    const int g = blockIdx.x - cb * a.n_groups;
    if (flags & kSplitInit) {
        split_init_state<16 * kNBF>(a, cb, g);
        return;
    }
    // The close of cycle t - 1 runs in workgroups of its own (after the row groups with kSplitRun, alone
    // without), beside the row groups that add cycle t's sums to the other slot.
    const int n_run = (flags & kSplitRun) ? a.n_cb * a.n_groups : 0;
    if ((int)blockIdx.x >= n_run) {
        if (flags & kSplitClose) split_close_cycle<16 * kNBF>(a, blockIdx.x - n_run, t - 1);
        return;
    }
    const bool update = (flags & kSplitUpdate) != 0;
    a.split_q = q_t;
    a.split_i0 = i0_t;
    a.t_begin = t;
    a.t_end = update ? t + 1 : t;
    a.final_pass = update ? 0 : 1;
    a.save_hist = 0;
    sweep_block<kFast, kMode, kNBF, kFp4, true>(a, cb, g);
}

// Many anneals in one launch: work item blockIdx.x is (anneal index << 16 | column block), listed by the
// host in decreasing cost so that the largest blocks start first.
template <bool kFast, int kMode, int kNBF, bool kFp4>
__global__ __launch_bounds__(kThreads, kNBF == 8 ? 1 : 2) void sweep_batch_kernel(const SweepArgs* __restrict__ items,
                                                                   const uint32_t* __restrict__ work) {
    const uint32_t w = work[blockIdx.x];
    const SweepArgs a = items[w >> 16];
    sweep_block<kFast, kMode, kNBF, kFp4>(a, (int)(w & 0xFFFFu));
}

// J [n][n] (int32, or int8 for a single-plane problem) -> P balanced int8 planes [P][np][np]
// (J = sum_p 256^p J_p), zero padded; also the padded h and the row sums of J.
template <typename TJ>
__global__ void prepare_planes_kernel(const TJ* J32, const int32_t* h32, int32_t n, int32_t np,
                                      int32_t P, int8_t* Jp, int32_t* rowvec) {
    const int i = blockIdx.x;
    if (i >= np) return;
    long long rs = 0;
    for (int j = threadIdx.x; j < np; j += blockDim.x) {
        int v = (i < n && j < n) ? (int)J32[(size_t)i * n + j] : 0;
        rs += v;
        const size_t off = tiled_offset(i, j, np);
        for (int p = 0; p < P; ++p) {
            const int8_t d = (int8_t)(v & 0xFF);
            Jp[(size_t)p * np * np + off] = d;
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
        const int32_t rs = (int32_t)part[0];
        const int32_t hv = i < n ? h32[i] : 0;
        rowvec[i] = hv;
        rowvec[np + i] = hv - rs;
        rowvec[2 * np + i] = 2 * hv - rs;
    }
}

// fp4 (e2m1) code of an integer coupling in {0, +-1, +-2, +-3, +-4, +-6}: magnitude codes 0, 2, 4, 5, 6, 7,
// sign in bit 3.
__device__ inline uint32_t fp4_code(int v) {
    const int m = v < 0 ? -v : v;
    const uint32_t c = m == 0 ? 0u : m == 1 ? 2u : m == 2 ? 4u : m == 3 ? 5u : m == 4 ? 6u : 7u;
    return (v < 0 && m != 0) ? (c | 8u) : c;
}

template <typename TJ>
__global__ void prepare_fp4_kernel(const TJ* J32, int32_t n, int32_t np, int32_t kp4, uint8_t* J4) {
    const int i = blockIdx.x;
    if (i >= np) return;
    for (int q = threadIdx.x; q < kp4 / 2; q += blockDim.x) {
        const int j0 = (q >> 4) * 32 + (q & 15);      // K offset with bit 4 clear; its partner is j0 + 16
        const int j1 = j0 + 16;
        const int v0 = (i < n && j0 < n) ? (int)J32[(size_t)i * n + j0] : 0;
        const int v1 = (i < n && j1 < n) ? (int)J32[(size_t)i * n + j1] : 0;
        int nib;
        const size_t off = tiled_offset_fp4(i, j0, kp4, &nib);
        J4[off] = (uint8_t)(fp4_code(v0) | (fp4_code(v1) << 4));
    }
}

// Public state -> internal layout, one workgroup per (trial, replica) column: counters of real spins
// (padded spins start at 0; they never reach a real spin) and the delayed bit planes in spread order.
__global__ void import_state_kernel(const int8_t* counters, const uint32_t* history, int32_t n, int32_t np,
                                    int32_t R, int32_t T, int32_t tpw, int32_t nb, int32_t delay, int8_t* is_state,
                                    uint32_t* hist_state) {
    const int col = blockIdx.x;   // b * R + k
    const int b = col / R;
    const int k = col - b * R;
    if (b >= T) return;
    const int wg = b / tpw;
    const int lc = (b - wg * tpw) * R + k;
    int8_t* dst = is_state + ((size_t)wg * nb + lc) * np;
    for (int i = threadIdx.x; i < np; i += blockDim.x) dst[i] = i < n ? counters[(size_t)col * n + i] : 0;
    const int words = np / 32, W = (n + 31) / 32;
    for (int u = threadIdx.x; u < delay * words; u += blockDim.x) {
        const int s = u / words;
        const int w = u - s * words;
        const uint32_t natural = w < W ? history[((size_t)col * delay + s) * W + w] : 0u;
        hist_state[(((size_t)wg * delay + s) * nb + lc) * words + w] = spread_bits(natural);
    }
}

// Internal delayed bit planes -> public history in natural bit order (bits past N cleared).
__global__ void export_history_kernel(const uint32_t* hist_state, int32_t n, int32_t np, int32_t R, int32_t T,
                                      int32_t tpw, int32_t nb, int32_t delay, uint32_t* history) {
    const int col = blockIdx.x;
    const int b = col / R;
    const int k = col - b * R;
    if (b >= T) return;
    const int wg = b / tpw;
    const int lc = (b - wg * tpw) * R + k;
    const int words = np / 32, W = (n + 31) / 32;
    for (int u = threadIdx.x; u < delay * W; u += blockDim.x) {
        const int s = u / W;
        const int w = u - s * W;
        const uint32_t spread = hist_state[(((size_t)wg * delay + s) * nb + lc) * words + w];
        uint32_t natural = 0;
        for (int o = 0; o < 32; ++o) natural |= ((spread >> bitpos(o)) & 1u) << o;
        const int valid = n - 32 * w;
        if (valid < 32) natural &= (1u << valid) - 1u;
        history[((size_t)col * delay + s) * W + w] = natural;
    }
}

__global__ void copy_final_is_kernel(const int8_t* is_state, int32_t np, int32_t n, int32_t R, int32_t T,
                                     int32_t tpw, int32_t nb, int8_t* out) {
    const int col = blockIdx.x;   // b * R + k
    const int b = col / R;
    const int k = col - b * R;
    if (b >= T) return;
    const int wg = b / tpw;
    const int lc = (b - wg * tpw) * R + k;
    const int8_t* src = is_state + ((size_t)wg * nb + lc) * np;
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
            const int8_t* plane = prob.J + (size_t)p * prob.np * prob.np;
            long long acc = 0;
            for (int j = 0; j < prob.n; ++j) acc += (int)plane[tiled_offset(i, j, prob.np)] * (int)s[j];
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

// QMC Hamiltonian (Eq. 4) of one trial per workgroup from its counters: sigma = +1 where Is >= 0.
// H_c = sum_k H_p(sigma_k) - J_perp sum_k sum_i sigma_{i,k} sigma_{i,k+1 mod R}.
__global__ void qmc_energy_kernel(DeviceProblem prob, const int8_t* counters, int32_t R, int32_t jperp,
                                  int64_t* out) {
    const int b = blockIdx.x;
    const int n = prob.n;
    const int8_t* trial = counters + (size_t)b * R * n;
    long long part = 0;   // accumulates -2 H_c
    for (int k = 0; k < R; ++k) {
        const int8_t* s = trial + (size_t)k * n;
        const int8_t* up = trial + (size_t)(k + 1 == R ? 0 : k + 1) * n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int si = s[i] >= 0 ? 1 : -1;
            long long F = 0;
            for (int p = prob.planes - 1; p >= 0; --p) {
                const int8_t* plane = prob.J + (size_t)p * prob.np * prob.np;
                long long acc = 0;
                for (int j = 0; j < n; ++j) acc += (int)plane[tiled_offset(i, j, prob.np)] * (s[j] >= 0 ? 1 : -1);
                F = F * 256 + acc;
            }
            part += (long long)si * (2LL * prob.h[i] + F);                 // -2 H_p contribution
            part += 2LL * jperp * si * (up[i] >= 0 ? 1 : -1);            // -2 (-J_perp sigma sigma_up)
        }
    }
    __shared__ long long red[256];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = -red[0] / 2;
}

}  // namespace

hipError_t launch_qmc_energy(const DeviceProblem& prob, const int8_t* counters, int32_t trials, int32_t R,
                             int32_t jperp, int64_t* out, hipStream_t stream) {
    hipLaunchKernelGGL(qmc_energy_kernel, dim3(trials), dim3(256), 0, stream, prob, counters, R, jperp, out);
    return hipGetLastError();
}

size_t split_lds_bytes(int np, int nb) {
    return (size_t)nb * (np / 32 + 1) * 4 + (size_t)2 * nb * kGroupWords * 4 + (size_t)kWaves * nb * 16 +
           (size_t)nb * 4 * 2 + (size_t)nb * 8 + (size_t)nb * 4 + (size_t)kWaves * 256 * 4;
}

size_t sweep_lds_bytes(int np, int delay, int nb) {
    const size_t plane_words = (size_t)nb * (np / 32 + 1);
    return (size_t)(delay + 2) * plane_words * 4 + (size_t)kWaves * nb * 16 + (size_t)nb * 4 * 2 + (size_t)nb * 8 +
           (size_t)nb * 4 + (size_t)kWaves * 256 * 4;
}

hipError_t launch_prepare_fp4(const void* J, int elem, int32_t n, int32_t np, int32_t kp4, uint8_t* J4,
                              hipStream_t stream) {
    if (elem == 1)
        hipLaunchKernelGGL(prepare_fp4_kernel<int8_t>, dim3(np), dim3(256), 0, stream, static_cast<const int8_t*>(J), n,
                           np, kp4, J4);
    else
        hipLaunchKernelGGL(prepare_fp4_kernel<int32_t>, dim3(np), dim3(256), 0, stream, static_cast<const int32_t*>(J),
                           n, np, kp4, J4);
    return hipGetLastError();
}

hipError_t launch_prepare_planes(const void* J, int elem, const int32_t* h32, int32_t n, int32_t np, int32_t planes,
                                 int8_t* Jp, int32_t* rowvec, hipStream_t stream) {
    if (elem == 1)
        hipLaunchKernelGGL(prepare_planes_kernel<int8_t>, dim3(np), dim3(256), 0, stream, static_cast<const int8_t*>(J),
                           h32, n, np, planes, Jp, rowvec);
    else
        hipLaunchKernelGGL(prepare_planes_kernel<int32_t>, dim3(np), dim3(256), 0, stream,
                           static_cast<const int32_t*>(J), h32, n, np, planes, Jp, rowvec);
    return hipGetLastError();
}

template <bool kFast, int kMode, int kNBF, bool kFp4>
hipError_t configure_variant() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_kernel<kFast, kMode, kNBF, kFp4>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_batch_kernel<kFast, kMode, kNBF, kFp4>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if constexpr (kNBF != 8) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_split_kernel<kFast, kMode, kNBF, kFp4>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }
    return e;
}

// Variant v < 16: bit 3 fast epilogue, bit 2 coupling mode 1, bit 1 fp4 operands, bit 0 32 columns per
// workgroup (else 64).  v = 16 .. 23: 128 columns; v = 16 .. 19 fp4 operands, 20 .. 23 int8 operands; bit 1
// fast epilogue, bit 0 coupling mode 1.
#define SSQA_FOR_EACH_VARIANT(X) \
    X(0, false, 0, 4, false) X(1, false, 0, 2, false) X(2, false, 0, 4, true) X(3, false, 0, 2, true) \
    X(4, false, 1, 4, false) X(5, false, 1, 2, false) X(6, false, 1, 4, true) X(7, false, 1, 2, true) \
    X(8, true, 0, 4, false) X(9, true, 0, 2, false) X(10, true, 0, 4, true) X(11, true, 0, 2, true) \
    X(12, true, 1, 4, false) X(13, true, 1, 2, false) X(14, true, 1, 4, true) X(15, true, 1, 2, true) \
    X(16, false, 0, 8, true) X(17, false, 1, 8, true) X(18, true, 0, 8, true) X(19, true, 1, 8, true) \
    X(20, false, 0, 8, false) X(21, false, 1, 8, false) X(22, true, 0, 8, false) X(23, true, 1, 8, false)

hipError_t configure_sweep_kernels() {
    static hipError_t status = [] {
        hipError_t e = hipSuccess;
#define SSQA_CONFIGURE(v, al, mo, nbf, f4) \
    if (e == hipSuccess) e = configure_variant<al, mo, nbf, f4>();
        SSQA_FOR_EACH_VARIANT(SSQA_CONFIGURE)
#undef SSQA_CONFIGURE
        return e;
    }();
    return status;
}

int sweep_variant(bool fast, int mode, int nb, bool fp4) {
    if (nb == 128) return (fp4 ? 16 : 20) + (fast ? 2 : 0) + (mode ? 1 : 0);
    return (fast ? 8 : 0) + (mode ? 4 : 0) + (fp4 ? 2 : 0) + (nb == 32 ? 1 : 0);
}

int variant_columns(int variant) { return variant >= 16 ? 128 : (variant & 1) ? 32 : 64; }

hipError_t launch_sweep_batch(const SweepArgs* items, const uint32_t* work, int n_work, int max_np, int max_delay,
                              int variant, hipStream_t stream) {
    const int nb = variant_columns(variant);
    const size_t lds = sweep_lds_bytes(max_np, max_delay, nb);
    const dim3 grid(n_work), block(kThreads);
    switch (variant) {
#define SSQA_LAUNCH_BATCH(v, al, mo, nbf, f4)                                                                \
    case v:                                                                                                \
        hipLaunchKernelGGL((sweep_batch_kernel<al, mo, nbf, f4>), grid, block, lds, stream, items, work); \
        break;
        SSQA_FOR_EACH_VARIANT(SSQA_LAUNCH_BATCH)
#undef SSQA_LAUNCH_BATCH
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep_split(const SweepArgs* item, const SweepArgs& host, int t, int flags, const int32_t* jperp,
                              const int32_t* i0, hipStream_t stream) {
    const int q_t = (flags & kSplitUpdate) ? jperp[t] : 0;
    const int i0_t = (flags & kSplitUpdate) ? i0[t] : 0;
    const hipError_t ce = configure_sweep_kernels();
    if (ce != hipSuccess) return ce;
    const size_t lds = (flags & kSplitRun) ? split_lds_bytes(host.prob.np, host.nb) +
                                                 (host.split_k == 4 ? split_k_lds_bytes(host.nb) : 0)
                                           : 0;
    // row groups (init, run), then one closing workgroup per column block (close)
    const int n_rows = (flags & (kSplitInit | kSplitRun)) ? host.n_cb * host.n_groups : 0;
    const int n_close = (flags & kSplitClose) && !(flags & kSplitInit) ? host.n_cb : 0;
    if (n_rows + n_close == 0) return hipSuccess;
    const dim3 grid(n_rows + n_close), block(kThreads);
    switch (sweep_variant(host.fast != 0, host.mode, host.nb, host.fp4 != 0)) {
#define SSQA_LAUNCH_SPLIT(v, al, mo, nbf, f4)                                                                   \
    case v:                                                                                                   \
        if constexpr (nbf != 8) {                                                                             \
            hipLaunchKernelGGL((sweep_split_kernel<al, mo, nbf, f4>), grid, block, lds, stream, item, t, flags, q_t, i0_t); \
            break;                                                                                            \
        } else {                                                                                              \
            return hipErrorInvalidValue;                                                                      \
        }
        SSQA_FOR_EACH_VARIANT(SSQA_LAUNCH_SPLIT)
#undef SSQA_LAUNCH_SPLIT
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs& a, int n_wg, hipStream_t stream) {
    const hipError_t ce = configure_sweep_kernels();
    if (ce != hipSuccess) return ce;
    const size_t lds = sweep_lds_bytes(a.prob.np, a.delay, a.nb);
    const dim3 grid(n_wg), block(kThreads);
    switch (sweep_variant(a.fast != 0, a.mode, a.nb, a.fp4 != 0)) {
#define SSQA_LAUNCH_ONE(v, al, mo, nbf, f4)                                                \
    case v:                                                                              \
        hipLaunchKernelGGL((sweep_kernel<al, mo, nbf, f4>), grid, block, lds, stream, a); \
        break;
        SSQA_FOR_EACH_VARIANT(SSQA_LAUNCH_ONE)
#undef SSQA_LAUNCH_ONE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_import_state(const int8_t* counters, const uint32_t* history, int32_t n, int32_t np, int32_t R,
                               int32_t T, int32_t tpw, int32_t nb, int32_t delay, int8_t* is_state,
                               uint32_t* hist_state, hipStream_t stream) {
    hipLaunchKernelGGL(import_state_kernel, dim3(T * R), dim3(256), 0, stream, counters, history, n, np, R, T, tpw,
                       nb, delay, is_state, hist_state);
    return hipGetLastError();
}

hipError_t launch_export_history(const uint32_t* hist_state, int32_t n, int32_t np, int32_t R, int32_t T,
                                 int32_t tpw, int32_t nb, int32_t delay, uint32_t* history, hipStream_t stream) {
    hipLaunchKernelGGL(export_history_kernel, dim3(T * R), dim3(256), 0, stream, hist_state, n, np, R, T, tpw, nb,
                       delay, history);
    return hipGetLastError();
}

hipError_t launch_copy_final_is(const int8_t* is_state, int32_t np, int32_t n, int32_t R, int32_t T, int32_t tpw,
                                int32_t nb, int8_t* out, hipStream_t stream) {
    hipLaunchKernelGGL(copy_final_is_kernel, dim3(T * R), dim3(256), 0, stream, is_state, np, n, R, T, tpw, nb, out);
    return hipGetLastError();
}

// Device state (counters, bit-plane history, schedules) of ssqa_anneal_noalloc, for callers that cannot
// allocate: a fixed array in the code object, one copy per device.  Host code never passes its name to a
// kernel (on the host the name is only a stand-in); it looks the device address up once per device with
// that device current and passes that address instead.
static __device__ __align__(256) uint8_t scratch[kFixedScratchBytes];

hipError_t fixed_scratch(int device, void** ptr) {
    static std::mutex lock;
    static void* addr[64] = {};
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_energy(const DeviceProblem& prob, const int8_t* spins, int32_t cols, int64_t* energies,
                         hipStream_t stream) {
    hipLaunchKernelGGL(energy_kernel, dim3(cols), dim3(256), 0, stream, prob, spins, cols, energies);
    return hipGetLastError();
}

}  // namespace ssqa
