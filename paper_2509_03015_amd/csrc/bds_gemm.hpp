// Work-group tile products for the per-level contractions (the trsm of the
// coupling blocks and the Schur updates of Alg. 3), staged through LDS.
//
// A work-group of 4 waves (2 x 2) accumulates an MT x MT output tile
// C += sum over terms of op(A_t) op(B_t); each wave owns an (MT/2) x (MT/2)
// sub-tile as (MT/32)^2 MFMA accumulator tiles.  The contraction index k runs
// over the terms one after the other in chunks of KC (16, or 32 for FP32 on
// large blocks): a chunk of both operands (MT x KC each) is loaded from global
// memory into registers while the previous chunk is multiplied out of LDS,
// then stored into the other LDS buffer (double buffering, one barrier per
// chunk).
//
// Operands are given as "rows x k" views: element (r, k) of a view is
// p[r * ld + k] when kc (k contiguous) or p[k * ld + r] otherwise.  A is
// viewed with its output row as r, B with its output column as r, so that
// C[m][n] += sum_k A(m, k) B(n, k).
#pragma once

#include <hip/hip_runtime.h>

#include "bds_chol.hpp"
#include "bds_device.hpp"

namespace bds {

template <typename T> struct View {
    const T* p;
    int64_t ld;
    bool kc;
};

// One term of a tile product: rows m0.. of A, rows n0.. of B, k in [k0, k1).
template <typename TA, typename TB> struct Term {
    View<TA> a;
    View<TB> b;
    int k0, k1;  // multiples of the chunk depth KC
};

// Depth KC of one K chunk: 16, or 32 for FP32 products on large blocks (their
// MFMAs take half the cycles per k step of FP64, so a deeper chunk keeps the
// work per barrier and the bytes in flight per work-group as for FP64; the
// launcher chooses).
template <typename T, int MT, int KC> struct GemmSmem {
    static constexpr int LD = KC + 16 / (int)sizeof(T);  // row stride: KC elements plus 16 bytes
    T a[2][MT * LD];
    T b[2][MT * LD];
};

// Elements per thread and operand of one chunk (MT x KC by 256 threads).
template <int MT, int KC> struct ChunkEpt { static constexpr int value = MT * KC / 256; };

// Global -> registers: the thread's share of rows [r0, r0 + MT) x k [k, k + KC).
template <typename V, int MT, int KC, typename T>
__device__ __forceinline__ void chunk_load(const View<T>& v, int r0, int k, V (&reg)[ChunkEpt<MT, KC>::value])
{
    constexpr int E = ChunkEpt<MT, KC>::value;
    const int t = threadIdx.x;
    if (v.kc) {
        // KC / E threads per row, E consecutive k each
        const int row = t / (KC / E), kk = (t % (KC / E)) * E;
        const T* src = v.p + (int64_t)(r0 + row) * v.ld + k + kk;
#pragma unroll
        for (int q = 0; q < E; ++q) reg[q] = (V)src[q];
    } else {
        // KC consecutive threads take the KC k of one group of E consecutive rows,
        // so that their transposed LDS writes below fall in consecutive banks
        const int kk = t % KC, row = (t / KC) * E;
        const T* src = v.p + (int64_t)(k + kk) * v.ld + r0 + row;
#pragma unroll
        for (int q = 0; q < E; ++q) reg[q] = (V)src[q];
    }
}

// Registers -> LDS (rows x KC, row stride LD), matching chunk_load's split.
template <int MT, int KC, typename V>
__device__ __forceinline__ void chunk_store(bool kc, V* dst, const V (&reg)[ChunkEpt<MT, KC>::value])
{
    constexpr int E = ChunkEpt<MT, KC>::value;
    constexpr int LD = GemmSmem<V, MT, KC>::LD;
    const int t = threadIdx.x;
    if (kc) {
        const int row = t / (KC / E), kk = (t % (KC / E)) * E;
#pragma unroll
        for (int q = 0; q < E; ++q) dst[row * LD + kk + q] = reg[q];
    } else {
        const int kk = t % KC, row = (t / KC) * E;
#pragma unroll
        for (int q = 0; q < E; ++q) dst[(row + q) * LD + kk] = reg[q];
    }
}

// Work skipped under a triangle: none; SKIP_TRI_B, term 0's B^T is lower
// triangular (column n of the output needs k <= n only); SKIP_SYM, the output
// tile is a diagonal tile of a symmetric matrix of which only the lower
// triangle is kept (16 x 16 tiles strictly above the diagonal are left out).
// With SKIP_SYM and sym set, every term is a Gram product (A and B are the
// same view and m0 == n0), so the B operand is read from A's LDS buffer and
// loaded only once.
enum { SKIP_NONE = 0, SKIP_TRI_B = 1, SKIP_SYM = 2 };

// Accumulator tiles (ta, tb), bit ta * R + tb, of wave (wm, wn) that take part.
template <int R> constexpr unsigned mask_cols_from(int tb0)
{
    unsigned m = 0;
    for (int ta = 0; ta < R; ++ta)
        for (int tb = tb0; tb < R; ++tb) m |= 1u << (ta * R + tb);
    return m;
}
template <int R> constexpr unsigned mask_lower(int w)
{
    unsigned m = 0;
    for (int ta = 0; ta < R; ++ta)
        for (int tb = 0; tb < R; ++tb)
            if ((w & 1) + 2 * tb <= (w >> 1) + 2 * ta) m |= 1u << (ta * R + tb);
    return m;
}

// Accumulate the terms into acc.  Wave (wm, wn) of the 2 x 2 arrangement owns
// the interleaved 16-row tiles wm, wm + 2, ... and 16-column tiles wn, wn + 2,
// ... of the MT x MT tile, so that work skipped under a triangle spreads over
// the waves.  With a SKIP mode a chunk runs one of a few straight MFMA
// sequences, chosen once per chunk (SKIP_TRI_B: the wave's first column tile
// with work left) or once per tile (SKIP_SYM, when sym is set: the wave's
// tiles on or below the diagonal); a branch per MFMA would break the
// accumulator chains apart.
template <typename C, int MT, int KC, int NTERM, int SKIP = SKIP_NONE, typename TA, typename TB>
__device__ __forceinline__ void wg_tile_product(typename AccT<C>::type (&acc)[MT / 32][MT / 32],
                                                const Term<TA, TB> (&terms)[NTERM], int m0, int n0,
                                                GemmSmem<typename Stor<C>::type, MT, KC>& sm, bool sym = false)
{
    using V = typename Stor<C>::type;
    constexpr int R = MT / 32;
    constexpr int E = ChunkEpt<MT, KC>::value;
    constexpr int LD = GemmSmem<V, MT, KC>::LD;
    static_assert(KC == 16 || KC == 32, "chunk depth 16 or 32");
    const int w = wave_id(), wm = w >> 1, wn = w & 1;
    const bool gram = SKIP == SKIP_SYM && sym;
    const int l = lane_id(), i = l & 15, g = l >> 4;

    static_assert(NTERM == 1 || NTERM == 2, "one or two terms");
    // chunk c -> (term, k): the chunks of term 0, then those of term 1
    const int nch0 = (terms[0].k1 - terms[0].k0) / KC;
    const int nch = nch0 + (NTERM == 2 ? (terms[NTERM - 1].k1 - terms[NTERM - 1].k0) / KC : 0);
    auto locate = [&](int c, int& t, int& k) {
        t = (NTERM == 2 && c >= nch0) ? 1 : 0;
        k = t == 0 ? terms[0].k0 + KC * c : terms[NTERM - 1].k0 + KC * (c - nch0);
    };
    // the term's views, chosen with selects (indexing the array with a run-time
    // index would put it in scratch memory)
    auto view_a = [&](int t) { return (NTERM == 2 && t) ? terms[NTERM - 1].a : terms[0].a; };
    auto view_b = [&](int t) { return (NTERM == 2 && t) ? terms[NTERM - 1].b : terms[0].b; };
    V ra[E], rb[E];
    if (nch == 0) return;
    {
        int t, k;
        locate(0, t, k);
        const View<TA> va = view_a(t);
        const View<TB> vb = view_b(t);
        chunk_load<V, MT, KC>(va, m0, k, ra);
        if (!gram) chunk_load<V, MT, KC>(vb, n0, k, rb);
        chunk_store<MT, KC>(va.kc, sm.a[0], ra);
        if (!gram) chunk_store<MT, KC>(vb.kc, sm.b[0], rb);
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        int t1 = 0, k1 = 0;
        bool kc_a = true, kc_b = true;
        if (c + 1 < nch) {
            locate(c + 1, t1, k1);
            const View<TA> va = view_a(t1);
            const View<TB> vb = view_b(t1);
            kc_a = va.kc;
            kc_b = vb.kc;
            chunk_load<V, MT, KC>(va, m0, k1, ra);
            if (!gram) chunk_load<V, MT, KC>(vb, n0, k1, rb);
        }
        const V* As = sm.a[c & 1] + (16 * wm + i) * LD + 4 * g;
        const V* Bs = (gram ? sm.a[c & 1] : sm.b[c & 1]) + (16 * wn + i) * LD + 4 * g;
        // MFMAs of 16 k of this chunk (from koff) for the accumulator tiles in MASK
        auto body = [&](auto mask_c, int koff) {
            constexpr unsigned MASK = decltype(mask_c)::value;
            auto on = [](int ta, int tb) { return ((MASK >> (ta * R + tb)) & 1u) != 0; };
            auto col_on = [&](int tb) {
                bool any = false;
                for (int ta = 0; ta < R; ++ta) any = any || on(ta, tb);
                return any;
            };
            if constexpr (std::is_same<C, bf16x>::value) {
                V a[R][4], b[R][4];
#pragma unroll
                for (int ta = 0; ta < R; ++ta) ld4(As + koff + 32 * ta * LD, a[ta]);
#pragma unroll
                for (int tb = 0; tb < R; ++tb)
                    if (col_on(tb)) ld4(Bs + koff + 32 * tb * LD, b[tb]);
#pragma unroll
                for (int ta = 0; ta < R; ++ta)
#pragma unroll
                    for (int tb = 0; tb < R; ++tb)
                        if (on(ta, tb)) tile_mac<C>(acc[ta][tb], a[ta], b[tb]);
            } else {
                // two k-steps at a time keeps the operand registers at 4 R
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    V a[R][2], b[R][2];
#pragma unroll
                    for (int ta = 0; ta < R; ++ta)
#pragma unroll
                        for (int q = 0; q < 2; ++q) a[ta][q] = As[koff + 32 * ta * LD + 2 * h + q];
#pragma unroll
                    for (int tb = 0; tb < R; ++tb)
                        if (col_on(tb))
#pragma unroll
                            for (int q = 0; q < 2; ++q) b[tb][q] = Bs[koff + 32 * tb * LD + 2 * h + q];
#pragma unroll
                    for (int q = 0; q < 2; ++q)
#pragma unroll
                        for (int ta = 0; ta < R; ++ta)
#pragma unroll
                            for (int tb = 0; tb < R; ++tb)
                                if (on(ta, tb)) acc[ta][tb] = mma(a[ta][q], b[tb][q], acc[ta][tb]);
                }
            }
        };
        using std::integral_constant;
        constexpr unsigned ALL = mask_cols_from<R>(0);
        static_assert(R <= 4, "at most four tiles per wave and direction");
        int tc = 0, kcur = 0;
        locate(c, tc, kcur);
#pragma unroll
        for (int koff = 0; koff < KC; koff += 16) {
            if constexpr (SKIP == SKIP_TRI_B) {
                // column tile wn + 2 tb needs the 16-k steps cr = (k - n0) / 16 <= wn + 2 tb
                const int cr = (kcur + koff - n0) >> 4;
                const int tb0 = (tc == 0 && cr > wn) ? (cr - wn + 1) >> 1 : 0;
                switch (tb0) {
                case 0: body(integral_constant<unsigned, ALL>{}, koff); break;
                case 1: body(integral_constant<unsigned, mask_cols_from<R>(1)>{}, koff); break;
                case 2: body(integral_constant<unsigned, mask_cols_from<R>(2)>{}, koff); break;
                case 3: body(integral_constant<unsigned, mask_cols_from<R>(3)>{}, koff); break;
                default: break;  // no column tile of this wave is reached yet
                }
            } else if constexpr (SKIP == SKIP_SYM) {
                switch (sym ? w : 4) {
                case 0: body(integral_constant<unsigned, mask_lower<R>(0)>{}, koff); break;
                case 1: body(integral_constant<unsigned, mask_lower<R>(1)>{}, koff); break;
                case 2: body(integral_constant<unsigned, mask_lower<R>(2)>{}, koff); break;
                case 3: body(integral_constant<unsigned, mask_lower<R>(3)>{}, koff); break;
                default: body(integral_constant<unsigned, ALL>{}, koff); break;
                }
            } else {
                body(integral_constant<unsigned, ALL>{}, koff);
            }
        }
        if (c + 1 < nch) {
            chunk_store<MT, KC>(kc_a, sm.a[(c + 1) & 1], ra);
            if (!gram) chunk_store<MT, KC>(kc_b, sm.b[(c + 1) & 1], rb);
        }
        __syncthreads();
    }
}

// Visit every element of the work-group tile owned by the calling wave:
// f(row, col, value) with the interleaved tile ownership of wg_tile_product.
template <typename C, int MT, typename F>
__device__ __forceinline__ void wg_tile_foreach(const typename AccT<C>::type (&acc)[MT / 32][MT / 32], int m0,
                                                int n0, F f)
{
    constexpr int R = MT / 32;
    const int w = wave_id(), wm = w >> 1, wn = w & 1;
    const int l = lane_id(), i = l & 15, g = l >> 4;
#pragma unroll
    for (int ta = 0; ta < R; ++ta)
#pragma unroll
        for (int tb = 0; tb < R; ++tb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                f(m0 + 16 * (wm + 2 * ta) + acc_row<C>(g, r), n0 + 16 * (wn + 2 * tb) + i, acc[ta][tb][r]);
}

// Map the launch's block index to a work index so that consecutive work
// indices run on the same XCD (blocks are dealt round-robin over the 8 XCDs),
// which keeps operands shared by neighbouring work items in one L2.
__device__ __forceinline__ int64_t xcd_local_index(int64_t bid, int64_t nblocks)
{
    const int64_t xcd = bid & 7, idx = bid >> 3;
    const int64_t per = nblocks >> 3, rem = nblocks & 7;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

}  // namespace bds
