// Register-resident Cholesky factorisation and triangular inversion of one
// np x np SPD block by one work-group (the potrf of the paper's Alg. 1/4,
// followed by the explicit inverse that lets every later triangular solve be
// a product).
//
// Layout.  The block is cut into 16 x 16 tiles; the nt(nt+1)/2 tiles of the
// lower triangle are dealt round-robin to the W waves of the work-group, and
// each wave keeps its tiles in MFMA accumulator registers for the whole call.
// A tile's register slot first holds A[I][K]; at panel K it becomes the tile
// L[I][K] of the Cholesky factor, which is published to LDS and then dropped,
// and the slot restarts as the tile X[I][K] of the inverse X = L^-1 (zero,
// then updated by the panels K..I-1), which is finished and written out at
// panel I.  So the inverse costs no extra registers.
//
// Right-looking sweep over the tile columns J = 0 .. nt-1 (one panel each):
//   1  owners publish A[J][J] (pivot tile), A[I][J] (I > J) and the
//      accumulated right-hand sides R[J][K] (K < J) to LDS;
//   2  one wave factorises the pivot tile in registers (16 lanes, one column
//      each, cross-lane reads) and inverts it: D = L[J][J]^-1;
//   3  L[I][J] = A[I][J] D^T and X[J][K] = D R[J][K] (MFMA), X[J][K] and
//      X[J][J] = D written to the output;
//   4  trailing updates A[I][K] -= L[I][J] L[K][J]^T (I >= K > J) and
//      R[I][K] -= L[I][J] X[J][K] (I > J >= K).
// The forward substitution L X = I carried along in step 4 is what makes
// X = L^-1.  The panel buffer holds nt tiles: slots I > J carry column J of
// L and slots K <= J carry row J of X (stored transposed), which never
// overlap.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "bds_device.hpp"

namespace bds {

// Row stride of a staged 16 x 16 tile: 16 elements plus 16 bytes, so that the
// 16-byte operand reads of the 16 lanes of a row group fall in distinct banks.
template <typename T> struct TileLd { static constexpr int value = 16 + 16 / (int)sizeof(T); };

template <typename T, int NT> struct CholSmem {
    static constexpr int LD = TileLd<T>::value;
    T pan[NT][16 * LD];  // column panel of L / row panel of X^T
    // pivot tiles, double-buffered by panel parity: the pivot of panel J + 1 is
    // factorised while panel J is still being used
    T dg[2][16 * LD];    // pivot tile (symmetric)
    T di[2][16 * LD];    // D = inverse of the pivot's Cholesky factor, row-major
    T dt[2][16 * LD];    // D^T, row-major
    int bad;
    int ready;           // last panel whose pivot tile has been staged
};

// Compute waves per work-group for a tile bound NT; the work-group has one
// more wave, the pivot wave, so it runs 64 (W + 1) threads.  Blocks of one or
// two tile columns (at most three tiles) get a single compute wave, so that
// twice as many work-groups fit on a CU; up to NT = 8 the work-group is 4
// waves, one per SIMD, so that several work-groups share a CU (waves are
// dealt to the SIMDs round-robin).
template <int NT> struct CholWaves { static constexpr int value = NT <= 2 ? 1 : (NT <= 8 ? 3 : 15); };
template <int NT> constexpr int chol_threads() { return 64 * (CholWaves<NT>::value + 1); }

// Value of lane R of each 16-lane row, broadcast to the whole row (DPP
// row_newbcast), kept in vector registers.  A double moves in one 64-bit DPP
// move (v_mov_b64 with row_newbcast), not as two 32-bit halves.
template <int R> __device__ __forceinline__ float row_bcast(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + R, 0xF, 0xF, true));
}
template <int R> __device__ __forceinline__ double row_bcast(double v)
{
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + R, 0xF, 0xF, true);
}

// Four consecutive elements starting at p (16-byte aligned for float, 32 for double).
template <typename T> __device__ __forceinline__ void ld4(const T* p, T (&v)[4])
{
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = p[s];
}

// acc += A B for one 16 x 16 x 16 tile product, with the A rows given as
// a[] = A[i][4g .. 4g+3] and the B columns as b[] = B[4g .. 4g+3][i]
// (lane l = 16 g + i), in the compute precision C.
template <typename C>
__device__ __forceinline__ void tile_mac(typename AccT<C>::type& acc, const typename Stor<C>::type (&a)[4],
                                         const typename Stor<C>::type (&b)[4])
{
    if constexpr (std::is_same<C, bf16x>::value) {
        sx4 ab, bb;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            ab[s] = bf16_bits(a[s]);
            bb[s] = bf16_bits(b[s]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ab, bb, acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = mma(a[s], b[s], acc);
    }
}

// acc (+)= sgn * P Q^T where P and Q are staged 16 x 16 tiles (row-major,
// stride LD): operand rows P[i][4g..] and Q[i][4g..].
template <typename C, int LD>
__device__ __forceinline__ void tile_mac_pqt(typename AccT<C>::type& acc, const typename Stor<C>::type* P,
                                             const typename Stor<C>::type* Q, bool negate)
{
    using T = typename Stor<C>::type;
    const int l = lane_id(), i = l & 15, g = l >> 4;
    T a[4], b[4];
    ld4(P + i * LD + 4 * g, a);
    ld4(Q + i * LD + 4 * g, b);
    if (negate) {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = -a[s];
    }
    tile_mac<C>(acc, a, b);
}

// Store an accumulator tile to a staged tile: row-major (transpose = false)
// or transposed.
template <typename C, int LD>
__device__ __forceinline__ void tile_stage(const typename AccT<C>::type& acc, typename Stor<C>::type* dst,
                                           bool transpose)
{
    const int l = lane_id(), i = l & 15, g = l >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = acc_row<C>(g, r);
        if (transpose)
            dst[i * LD + row] = acc[r];
        else
            dst[row * LD + i] = acc[r];
    }
}

// Store an accumulator tile to global memory (row-major, leading dimension ld).
template <typename C>
__device__ __forceinline__ void tile_store(const typename AccT<C>::type& acc, typename Stor<C>::type* dst,
                                           int64_t ld)
{
    const int l = lane_id(), i = l & 15, g = l >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(int64_t)acc_row<C>(g, r) * ld + i] = acc[r];
}

// Empty asm that the optimiser must assume redefines v: it pins the
// program order of the unrolled pivot steps below, so that each step's
// broadcasts are made and consumed inside that step (left to itself the
// compiler hoists all ~120 broadcasts of the sweep and runs out of registers).
template <typename T> __device__ __forceinline__ void pin(T& v) { asm volatile("" : "+v"(v)); }

// Column step k of the pivot factorisation: lane c of each row of 16 lanes
// holds column c of the working matrix in a[]; a[k] is replaced by L[c][k],
// so that a[] ends up holding row c of the factor, and lane k keeps
// rv = 1 / L[k][k].
template <typename T, int K>
__device__ __forceinline__ void pivot_chol_step(T (&a)[16], T& rv, int c, int& bad)
{
    pin(a[K]);
    const T piv = row_bcast<K>(a[K]);
    if (!(piv > (T)0) && bad < 0) bad = K;
    const T rinv = rsqrt(piv);
    const T lck = a[K] * rinv;  // L[c][k]
    a[K] = lck;
    if (c == K) rv = rinv;
    [&]<int... R>(std::integer_sequence<int, R...>) {
        ((a[K + 1 + R] -= row_bcast<K + 1 + R>(lck) * lck), ...);
    }(std::make_integer_sequence<int, 15 - K>{});
}

// Step k of the forward substitution L X = I for column c of X (lane c of
// each row of 16 lanes): x[k] /= L[k][k], then x[r] -= L[r][k] x[k] for
// r > k.  Row r of L is held by lane r (a[] after the factorisation, rv its
// reciprocal pivot), so its entries arrive by row broadcast.  The broadcasts
// do not depend on x, so the compiler prepares them ahead of the chain; for
// doubles the sources are pinned every second step, which bounds that
// look-ahead to two steps (about 60 registers) instead of the whole sweep.
template <typename T, int K>
__device__ __forceinline__ void pivot_inv_step(const T (&a)[16], T rv, T (&x)[16])
{
    pin(x[K]);
    T aK = a[K], rk = rv;
    if constexpr (sizeof(T) == 8 && K % 2 == 0) {
        pin(aK);
        pin(rk);
    }
    const T xk = x[K] * row_bcast<K>(rk);
    x[K] = xk;
    [&]<int... R>(std::integer_sequence<int, R...>) {
        ((x[K + 1 + R] -= row_bcast<K + 1 + R>(aK) * xk), ...);
    }(std::make_integer_sequence<int, 15 - K>{});
}

// Factorise the 16 x 16 symmetric pivot tile of panel J, staged in
// sm.dg[J & 1], and invert the factor: sm.di[J & 1] = L^-1 and
// sm.dt[J & 1] = (L^-1)^T (both row-major), by the calling wave.  The
// factorisation keeps column c of the working matrix in lane c of each row
// of 16 lanes (the four rows compute the same values) and leaves row c of L
// there; the forward substitution L X = I then gives lane c column c of
// X = L^-1, taking the entries of L by row broadcast from the lanes that hold
// them, all in registers.  Records the first non-positive pivot (column
// 16 J + k) in sm.bad.
template <typename T, int NT>
__device__ __forceinline__ void pivot_factor(CholSmem<T, NT>& sm, int J)
{
    constexpr int LD = TileLd<T>::value;
    const int l = lane_id(), c = l & 15, b = J & 1;
    const T* dg = sm.dg[b];
    T a[16], rv = (T)0;
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = dg[r * LD + c];
    int bad = -1;
    [&]<int... K>(std::integer_sequence<int, K...>) { (pivot_chol_step<T, K>(a, rv, c, bad), ...); }(
        std::make_integer_sequence<int, 16>{});
    if (l == 0 && bad >= 0 && sm.bad < 0) sm.bad = 16 * J + bad;
    T x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = (r == c) ? (T)1 : (T)0;
    [&]<int... K>(std::integer_sequence<int, K...>) { (pivot_inv_step<T, K>(a, rv, x), ...); }(
        std::make_integer_sequence<int, 16>{});
    if (l < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            sm.di[b][r * LD + c] = x[r];
            sm.dt[b][c * LD + r] = x[r];
        }
    }
}

// Row panel J of the inverse (16 x np, row stride ldl) to global memory, by
// all WB waves of the work-group: wave w writes rows w, w + WB, ..., each lane
// two adjacent columns.  X[J][K] for K < J comes from the transposed tiles in
// sm.pan, X[J][J] from sm.di[J & 1], and the tiles right of the diagonal are
// zero.
template <typename T, int NT, int WB>
__device__ __forceinline__ void store_row_panel(const CholSmem<T, NT>& sm, T* Li, int np, int64_t ldl, int J,
                                                int w)
{
    constexpr int LD = TileLd<T>::value;
    const int l = lane_id();
    for (int r = w; r < 16; r += WB) {
        T* dst = Li + (int64_t)(16 * J + r) * ldl;
        for (int c0 = 2 * l; c0 < np; c0 += 128) {
            const int K = c0 >> 4, c = c0 & 15;
            T v0 = (T)0, v1 = (T)0;
            if (K < J) {
                v0 = sm.pan[K][c * LD + r];
                v1 = sm.pan[K][(c + 1) * LD + r];
            } else if (K == J) {
                v0 = sm.di[J & 1][r * LD + c];
                v1 = sm.di[J & 1][r * LD + c + 1];
            }
            dst[c0] = v0;
            dst[c0 + 1] = v1;
        }
    }
}

// Tile (I, K), I >= K, of lower-triangle index t = I (I + 1) / 2 + K.
__device__ __forceinline__ void tile_of(int t, int& I, int& K)
{
    int r = 0;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    I = r;
    K = t - r * (r + 1) / 2;
}

// Cholesky factor and inverse of one np x np block by the whole work-group
// (np = 16 nt, nt <= NT).  Waves 0 .. W-1 own the register tiles and run the
// tile products; wave W, which owns no tiles, factorises the pivot tiles (so
// that the registers of that serial step do not add to those of the tiles)
// one panel ahead: the owner of tile (J+1, J+1) updates it first in step 4 of
// panel J, stages it and raises sm.ready, and the pivot wave factorises it
// while the other waves finish panel J.
//   A  (np x np, element type In, row-major, row stride lda): only the lower
//      triangle is read;
//   Li (np x np, storage of C, row-major, row stride ldl): receives L^-1
//      (lower triangular, explicit zeros above the diagonal).
// Returns the first column whose pivot is not positive (or NaN), else -1.
template <typename C, int NT, int W, typename In>
__device__ __forceinline__ int chol_inv_block(const In* A, typename Stor<C>::type* Li, int np, int64_t lda,
                                              int64_t ldl, CholSmem<typename Stor<C>::type, NT>& sm)
{
    using T = typename Stor<C>::type;
    using Acc = typename AccT<C>::type;
    constexpr int LD = TileLd<T>::value;
    constexpr int S = (NT * (NT + 1) / 2 + W - 1) / W;  // register slots per compute wave
    const int nt = np >> 4;
    const int ntl = nt * (nt + 1) / 2;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = lane_id(), i = l & 15, g = l >> 4;
    if (threadIdx.x == 0) {
        sm.bad = -1;
        sm.ready = 0;
    }

    if (w == W) {
        // pivot wave
        __syncthreads();  // pivot tile of panel 0 staged
        pivot_factor<T, NT>(sm, 0);
        __syncthreads();
        for (int J = 0; J < nt; ++J) {
            __syncthreads();  // 1: panels published
            __syncthreads();  // 3: column J of L and row J of the inverse staged
            store_row_panel<T, NT, W + 1>(sm, Li, np, ldl, J, w);
            if (J + 1 < nt) {
                // wait for the owner of tile (J+1, J+1) to stage it (it does so
                // first thing in step 4, so the wait ends)
                while (__hip_atomic_load(&sm.ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < J + 1)
                    __builtin_amdgcn_s_sleep(1);
                pivot_factor<T, NT>(sm, J + 1);
            }
            __syncthreads();  // 4
        }
        return sm.bad;
    }

    // compute waves: tile coordinates of the register slots (wave-uniform)
    int tI[S], tK[S];
#pragma unroll
    for (int s = 0; s < S; ++s) tile_of(w + s * W, tI[s], tK[s]);

    // load the lower tiles, symmetric completion inside the diagonal tiles
    Acc acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int t = w + s * W;
        acc[s] = Acc{0, 0, 0, 0};
        if (t < ntl) {
            const int I = tI[s], K = tK[s];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = acc_row<C>(g, r);
                const int gr = 16 * I + row, gc = 16 * K + i;
                acc[s][r] = (T)((I == K && i > row) ? A[(int64_t)gc * lda + gr] : A[(int64_t)gr * lda + gc]);
            }
            if (I == 0 && K == 0) tile_stage<C, LD>(acc[s], sm.dg[0], false);
        }
    }
    __syncthreads();  // pivot tile of panel 0 staged
    __syncthreads();  // D of panel 0 ready

    for (int J = 0; J < nt; ++J) {
        const int b = J & 1;
        // 1: publish column J of A and row J of the right-hand sides
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int t = w + s * W;
            if (t >= ntl) continue;
            const int I = tI[s], K = tK[s];
            if (K == J && I > J)
                tile_stage<C, LD>(acc[s], sm.pan[I], false);
            else if (I == J && K < J)
                tile_stage<C, LD>(acc[s], sm.pan[K], true);
        }
        __syncthreads();  // 1
        // 3: L[I][J] = A[I][J] D^T; X[J][K] = D R[J][K]
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int t = w + s * W;
            if (t >= ntl) continue;
            const int I = tI[s], K = tK[s];
            if (K == J && I > J) {
                Acc p = Acc{0, 0, 0, 0};
                tile_mac_pqt<C, LD>(p, sm.pan[I], sm.di[b], false);
                tile_stage<C, LD>(p, sm.pan[I], false);
                acc[s] = Acc{0, 0, 0, 0};  // the slot restarts as the right-hand side R[I][J]
            } else if (I == J && K < J) {
                Acc p = Acc{0, 0, 0, 0};
                tile_mac_pqt<C, LD>(p, sm.di[b], sm.pan[K], false);
                tile_stage<C, LD>(p, sm.pan[K], true);
            }
        }
        __syncthreads();  // 3
        // 4: the next pivot tile first, then the row panel of the inverse and
        //    the other trailing updates
        //    A[I][K] -= L[I][J] L[K][J]^T (I >= K > J), R[I][K] -= L[I][J] X[J][K] (I > J >= K)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int t = w + s * W;
            if (t >= ntl) continue;
            const int I = tI[s], K = tK[s];
            if (I == J + 1 && K == J + 1) {
                tile_mac_pqt<C, LD>(acc[s], sm.pan[I], sm.pan[K], true);
                tile_stage<C, LD>(acc[s], sm.dg[(J + 1) & 1], false);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (l == 0) __hip_atomic_store(&sm.ready, J + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        store_row_panel<T, NT, W + 1>(sm, Li, np, ldl, J, w);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int t = w + s * W;
            if (t >= ntl) continue;
            const int I = tI[s], K = tK[s];
            if (I > J && !(I == J + 1 && K == J + 1))
                tile_mac_pqt<C, LD>(acc[s], sm.pan[I], K == J ? sm.dt[b] : sm.pan[K], true);
        }
        __syncthreads();  // 4
    }
    return sm.bad;
}

}  // namespace bds
