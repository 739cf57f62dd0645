// Device-side building blocks for gfx950: the MFMA wave-tile engine.
//
// MFMA conventions (v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32, wave64):
// for lane l let i = l % 16 and g = l / 16.  One instruction multiplies a
// 16 x 4 A fragment (lane l holds A[i][g]) by a 4 x 16 B fragment (lane l
// holds B[g][j=i]) into a 16 x 16 accumulator where lane l holds four rows
// of column i (which four: see acc_row below).  The engine walks K in chunks of 16 and feeds k-step
// s of a chunk with k = 4g + s, so that each lane reads four consecutive k
// (a vector load when the operand is contiguous along k); A and B use the same
// order, so every product term is summed exactly once.
//
// Accumulator layouts differ between the instructions: the FP32 and BF16 forms
// give lane l rows 4g .. 4g+3 of column i (register r -> row 4g + r), whereas
// the FP64 form interleaves them (register r -> row g + 4r).  acc_row() holds
// this mapping; every read of an accumulator goes through acc_foreach.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/bds.h"

namespace bds {

constexpr int kMaxNP = 256;  // largest padded block size

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));
typedef short sx4 __attribute__((ext_vector_type(4)));

// Compute tags.  double and float compute in their own precision; bf16x
// stores FP32 but rounds every MFMA operand to bfloat16 (round to nearest
// even) and accumulates in FP32 (v_mfma_f32_16x16x16_bf16).
struct bf16x {};

template <typename C> struct Stor { using type = C; };
template <> struct Stor<bf16x> { using type = float; };

template <typename T> struct AccT;
template <> struct AccT<double> { using type = dx4; };
template <> struct AccT<float> { using type = fx4; };
template <> struct AccT<bf16x> { using type = fx4; };
// The library's precision code (BDS_F64, BDS_F32, BDS_BF16) of a compute tag.
template <typename C> struct PrecOf { static constexpr int value = 0; };
template <> struct PrecOf<float> { static constexpr int value = 1; };
template <> struct PrecOf<bf16x> { static constexpr int value = 2; };

// FP32 -> bfloat16 bits, round to nearest even; NaN stays NaN.
__device__ __forceinline__ short bf16_bits(float x)
{
    const unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (short)0x7fc0;
    return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ dx4 mma(double a, double b, dx4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fx4 mma(float a, float b, fx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
// wave index within the work-group, as a wave-uniform (scalar) value
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

template <typename T, int RM, int RN>
__device__ __forceinline__ void acc_zero(typename AccT<T>::type (&acc)[RM][RN])
{
#pragma unroll
    for (int a = 0; a < RM; ++a)
#pragma unroll
        for (int b = 0; b < RN; ++b) acc[a][b] = typename AccT<T>::type{0, 0, 0, 0};
}

// Operand orientation.
//   A (M x K): A_MK -> element (m,k) at A[m*lda + k];  otherwise at A[k*lda + m].
//   B (K x N): B_NK -> element (k,n) at B[n*ldb + k];  otherwise at B[k*ldb + n].
// B_MASK: columns n >= ncols of B read as zero (right-hand sides with d < 16).
// acc[a][b] accumulates the 16 x 16 output tile (m0 + 16a, n0 + 16b).
// k0, k1: multiples of 16.
// UNR: k-steps whose loads are issued together before their products, so
// that a wave has UNR steps in flight (launches too small to hide load
// latency with other waves).
template <typename T, int RM, int RN, bool A_MK, bool B_NK, bool B_MASK = false, int UNR = 1, typename SA,
          typename SB>
__device__ __forceinline__ void wave_mma(typename AccT<T>::type (&acc)[RM][RN], const SA* A,
                                         int64_t lda, const SB* B, int64_t ldb, int m0, int n0,
                                         int k0, int k1, int ncols = 1 << 30)
{
    using V = typename Stor<T>::type;
    const int l = lane_id();
    const int i = l & 15, g = l >> 4;
    int kc = k0;
    // FP32 rows feeding FP64 products (solves with a low-precision factor): 32 k per
    // step, so that each lane reads 32 contiguous bytes of A as an FP64 row does;
    // lane group g takes k = 8g .. 8g+7 of the 32, for A and B alike
    constexpr bool WIDE = std::is_same<T, double>::value && sizeof(SA) == 4 && A_MK;
    constexpr int KS = WIDE ? 8 : 4;  // k per lane and step
    // operands of one step at kc (lane group g: k = kc + KS g ..)
    auto load = [&](int kc_, V (&a)[RM][KS], V (&b)[RN][KS]) {
        const int k = kc_ + KS * g;
#pragma unroll
        for (int ta = 0; ta < RM; ++ta) {
            const int m = m0 + 16 * ta + i;
#pragma unroll
            for (int s = 0; s < KS; ++s)
                a[ta][s] = A_MK ? (V)A[(int64_t)m * lda + k + s] : (V)A[(int64_t)(k + s) * lda + m];
        }
#pragma unroll
        for (int tb = 0; tb < RN; ++tb) {
            const int n = n0 + 16 * tb + i;
            const bool ok = !B_MASK || n < ncols;
#pragma unroll
            for (int s = 0; s < KS; ++s)
                b[tb][s] = ok ? (B_NK ? (V)B[(int64_t)n * ldb + k + s] : (V)B[(int64_t)(k + s) * ldb + n])
                              : (V)0;
        }
    };
    auto multiply = [&](const V (&a)[RM][KS], const V (&b)[RN][KS]) {
        if constexpr (std::is_same<T, bf16x>::value) {
            // one 16x16x16 instruction covers the four k-steps: lane (i, g) supplies k = 4g .. 4g+3
            sx4 ab[RM], bb[RN];
#pragma unroll
            for (int ta = 0; ta < RM; ++ta)
#pragma unroll
                for (int s = 0; s < 4; ++s) ab[ta][s] = bf16_bits(a[ta][s]);
#pragma unroll
            for (int tb = 0; tb < RN; ++tb)
#pragma unroll
                for (int s = 0; s < 4; ++s) bb[tb][s] = bf16_bits(b[tb][s]);
#pragma unroll
            for (int ta = 0; ta < RM; ++ta)
#pragma unroll
                for (int tb = 0; tb < RN; ++tb)
                    acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ab[ta], bb[tb], acc[ta][tb], 0, 0, 0);
        } else {
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int ta = 0; ta < RM; ++ta)
#pragma unroll
                    for (int tb = 0; tb < RN; ++tb) acc[ta][tb] = mma(a[ta][s], b[tb][s], acc[ta][tb]);
        }
    };
    constexpr int KSTEP = 4 * KS;  // k per step: 16, or 32 on the WIDE path
    if constexpr (UNR > 1) {
        // UNR steps' loads first, then their products
        for (; kc + UNR * KSTEP <= k1; kc += UNR * KSTEP) {
            V a[UNR][RM][KS], b[UNR][RN][KS];
#pragma unroll
            for (int u = 0; u < UNR; ++u) load(kc + u * KSTEP, a[u], b[u]);
#pragma unroll
            for (int u = 0; u < UNR; ++u) multiply(a[u], b[u]);
        }
    }
    for (; kc + KSTEP <= k1; kc += KSTEP) {
        V a[RM][KS], b[RN][KS];
        load(kc, a, b);
        multiply(a, b);
    }
    if constexpr (WIDE) {
        // a last 16 k in 16-k steps (k1 - k0 is a multiple of 16)
        for (; kc < k1; kc += 16) {
            const int k = kc + 4 * g;
            V a[RM][4], b[RN][4];
#pragma unroll
            for (int ta = 0; ta < RM; ++ta) {
                const int m = m0 + 16 * ta + i;
#pragma unroll
                for (int s = 0; s < 4; ++s) a[ta][s] = (V)A[(int64_t)m * lda + k + s];
            }
#pragma unroll
            for (int tb = 0; tb < RN; ++tb) {
                const int n = n0 + 16 * tb + i;
                const bool ok = !B_MASK || n < ncols;
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    b[tb][s] = ok ? (B_NK ? (V)B[(int64_t)n * ldb + k + s] : (V)B[(int64_t)(k + s) * ldb + n])
                                  : (V)0;
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int ta = 0; ta < RM; ++ta)
#pragma unroll
                    for (int tb = 0; tb < RN; ++tb) acc[ta][tb] = mma(a[ta][s], b[tb][s], acc[ta][tb]);
        }
    }
}

// Row within a 16 x 16 accumulator tile of register r in lane group g.
template <typename T> __device__ __forceinline__ int acc_row(int g, int r)
{
    return std::is_same<T, double>::value ? g + 4 * r : 4 * g + r;
}

// Visit every element of a wave's accumulator tile: f(row, col, value).
template <typename T, int RM, int RN, typename F>
__device__ __forceinline__ void acc_foreach(const typename AccT<T>::type (&acc)[RM][RN], int m0,
                                            int n0, F f)
{
    const int l = lane_id();
    const int i = l & 15, g = l >> 4;
#pragma unroll
    for (int ta = 0; ta < RM; ++ta)
#pragma unroll
        for (int tb = 0; tb < RN; ++tb)
#pragma unroll
            for (int r = 0; r < 4; ++r) f(m0 + 16 * ta + acc_row<T>(g, r), n0 + 16 * tb + i, acc[ta][tb][r]);
}

__device__ __forceinline__ void report_notspd(bds_info* info, int level, int pos, int orig, int col)
{
    if (!info) return;
    if (atomicCAS(&info->status, 0, (int)BDS_ENOTSPD) == 0) {
        info->level = level;
        info->position = pos;
        info->orig_block = orig;
        info->column = col;
    }
}

}  // namespace bds
