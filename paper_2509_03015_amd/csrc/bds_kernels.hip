// gfx950 kernels of the recursive Schur-complement solver.
//
// Per reduction level (the paper's Alg. 4 with segment length 1):
//   k_fac_diag    Li[e] = chol(A_ii)^-1 for every interior i = 2e+1
//                 (potrf followed by an explicit triangular inverse)
//   k_fac_couple  Wt[e] = A_{i-1,i} Li[e]^T,  Pr[e] = A_{i+1,i} Li[e]^T
//                 (the trsm of the coupling blocks, Alg. 4, as MFMA products;
//                 the left coupling Li A_{i,i-1} is kept transposed, as Wt, so
//                 that every Schur product below reads both operands along
//                 contiguous rows)
//   k_fac_schur   next level S (eq. (5), Alg. 3), one record per separator j:
//                 S_jj      = A_{2j,2j} - Pr[j-1] Pr[j-1]^T - Wt[j] Wt[j]^T
//                 S_{j+1,j} = -Pr[j] Wt[j]^T
//   k_coarse_factor  sequential block Cholesky of the coarse system (FP64).
// Per solve level (Alg. 5-7):
//   k_sol_fwd_int  Y[e] = Li[e] B_i
//   k_sol_fwd_sep  B'_j = B_2j - Pr[j-1] Y[j-1] - Wt[j] Y[j]  (Alg. 5)
//   k_coarse_solve block forward/backward substitution of the coarse system
//   k_sol_bwd      X_i = Li[e]^T (Y[e] - Wt[e]^T X_{i-1} - Pr[e]^T X_{i+1})
//                  (Alg. 6 followed by the interior solve), separators copied
//                  from the coarser level (the final Assemble of Alg. 7).
// Each separator receives its two contributions in a fixed order, so results
// are deterministic (no atomics in the arithmetic).
#include <algorithm>
#include <atomic>

#include "bds_chol.hpp"
#include "bds_device.hpp"
#include "bds_gemm.hpp"
#include "bds_kernels.hpp"
#include "bds_trace.hpp"

namespace bds {

// ---------------------------------------------------------------------------
// tables

template <typename S> struct One {
    S s;
    int64_t total;
    __device__ __forceinline__ const S& get(int64_t u, int64_t& local) const
    {
        local = u;
        return s;
    }
};

template <typename S> struct Many {
    const S* s;
    const int64_t* start;  // K + 1 exclusive prefix sums; nullptr: one unit per record
    int K;
    int64_t total;
    __device__ __forceinline__ const S& get(int64_t u, int64_t& local) const
    {
        if (!start) {
            local = 0;
            return s[u];
        }
        int lo = 0, hi = K - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= u)
                lo = mid;
            else
                hi = mid - 1;
        }
        local = u - start[lo];
        return s[lo];
    }
};

int tile_r(int np) { return (np % 32 == 0) ? 2 : 1; }
// Library rule for the tile shapes.  Couplings and Schur updates of blocks that
// are a multiple of 64 run as work-group tile products; the macro tile depends
// on the compute precision: FP64 64 (four work-groups per CU keep enough HBM
// reads in flight); the FP32 and BF16 MFMAs take 1/2 and 1/8 the cycles of
// FP64 per k step, so a 64-wide tile spends relatively more time per chunk on
// loads, LDS staging and the barrier, and 128-wide tiles halve that overhead
// per flop where np allows: both products in BF16, the couplings in FP32
// (measured: the FP32 Schur update is faster with 64).  Other block sizes use
// wave tiles, 32 x 32 where they divide np.
static_assert(PrecOf<double>::value == BDS_F64 && PrecOf<float>::value == BDS_F32 &&
                  PrecOf<bf16x>::value == BDS_BF16,
              "precision codes of the compute tags");
static int wave_rule(int np) { return np % 32 == 0 ? BDS_TILE_W32 : BDS_TILE_W16; }
static int couple_rule(int np, int prec)
{
    if (np % 64) return wave_rule(np);
    return (prec != BDS_F64 && np % 128 == 0) ? BDS_TILE_G128 : BDS_TILE_G64;
}
static int schur_rule(int np, int prec)
{
    if (np % 64) return wave_rule(np);
    return (prec == BDS_BF16 && np % 128 == 0) ? BDS_TILE_G128 : BDS_TILE_G64;
}
static bool tile_fits(int code, int np)
{
    switch (code) {
    case BDS_TILE_W16: return true;
    case BDS_TILE_W32: return np % 32 == 0;
    case BDS_TILE_G64: return np % 64 == 0;
    case BDS_TILE_G128: return np % 128 == 0;
    default: return false;
    }
}
bool resolve_tiling(int np, int prec, int32_t tiles, Tiling& t)
{
    if (tiles & ~0xFFF) return false;
    const int c = tiles & 15, sc = (tiles >> 4) & 15, v = (tiles >> 8) & 15;
    t.couple = c ? c : couple_rule(np, prec);
    t.schur = sc ? sc : schur_rule(np, prec);
    t.sol = v ? v : wave_rule(np);
    return tile_fits(t.couple, np) && tile_fits(t.schur, np) && tile_fits(t.sol, np) &&
           (t.sol == BDS_TILE_W16 || t.sol == BDS_TILE_W32);
}
std::vector<int> tile_choices(int np, bool solve)
{
    std::vector<int> v;
    for (int code : {BDS_TILE_W16, BDS_TILE_W32, BDS_TILE_G64, BDS_TILE_G128})
        if (tile_fits(code, np) && (!solve || code <= BDS_TILE_W32)) v.push_back(code);
    return v;
}
static inline int wave_r(int code) { return code == BDS_TILE_W32 ? 2 : 1; }

static int64_t units_fac_couple_wg(int M, int np, int MT);
static int64_t units_fac_schur_wg(int M, int np, int MT);
int64_t units_fac_diag(int M) { return M / 2; }
int64_t units_fac_couple(int M, int np, int code)
{
    if (code >= BDS_TILE_G64) return units_fac_couple_wg(M, np, code == BDS_TILE_G128 ? 128 : 64);
    const int tp = np / (16 * wave_r(code));
    return (int64_t)(M / 2) * 2 * tp * tp;
}
int64_t units_fac_schur(int M, int np, int code)
{
    if (code >= BDS_TILE_G64) return units_fac_schur_wg(M, np, code == BDS_TILE_G128 ? 128 : 64);
    const int tp = np / (16 * wave_r(code));
    return (int64_t)((M + 1) / 2) * (tp * (tp + 1) / 2 + tp * tp);
}
static inline int dchunks(int d) { return (d + 15) / 16; }
int64_t units_sol_fwd_int(int M, int np, int d, int code)
{
    return (int64_t)(M / 2) * (np / (16 * wave_r(code))) * dchunks(d);
}
int64_t units_sol_fwd_sep(int M, int np, int d, int code)
{
    return (int64_t)((M + 1) / 2) * (np / (16 * wave_r(code))) * dchunks(d);
}
int64_t units_sol_bwd(int M, int d) { return (int64_t)(M / 2) * dchunks(d); }
int64_t units_resid(int N, int np, int d) { return (int64_t)N * (np / (16 * tile_r(np))) * dchunks(d); }

// ---------------------------------------------------------------------------
// factorisation

// Four work-groups per CU for blocks up to 64 rows, two up to 128 (four or two
// waves per SIMD).  W
// compute waves (the default, CholWaves) or, on levels with fewer interiors
// than CUs, kWideWaves: one work-group per CU then, and the trailing updates
// of every panel spread over 15 waves (three register tiles each for a
// 128-row block) instead of three; the pivot chain is the same.
constexpr int kWideWaves = 15;

template <typename C, typename In, int NT, int W, typename Tab>
__global__ __launch_bounds__(64 * (W + 1))
__attribute__((amdgpu_waves_per_eu(NT <= 4 && W <= 3 ? 4 : (NT <= 8 && W <= 3 ? 2 : 1)))) void k_fac_diag(Tab tab)
{
    using T = typename Stor<C>::type;
    __shared__ CholSmem<T, NT> sm;
    const int64_t u = blockIdx.x;
    if (u >= tab.total) return;
    int64_t e;
    const auto& s = tab.get(u, e);
    const int np = s.np;
    const int64_t nn = (int64_t)np * np;
    const int64_t i = 2 * e + 1;
    const int bad = chol_inv_block<C, NT, W, In>(s.Ad + i * nn, s.Li + e * nn, np, np, np, sm);
    if (bad >= 0 && threadIdx.x == 0)
        report_notspd(s.info, s.level, (int)i, (int)(i << s.level), bad);
}

// FP64 blocks of 256 rows: the factor and inverse of A_ii by a 2 x 2 block
// recursion over 128-row halves, so that the serial pivot chains run in the
// 128-row kernel (several work-groups per CU) instead of one 16-wave
// work-group per CU:
//   L11^-1 = chol(A11)^-1               (k_fac_diag_half, first)
//   L21 = A21 L11^-T                    (k_fac_diag_link, step 0)
//   S = A22 - L21 L21^T                 (step 1)
//   L22^-1 = chol(S)^-1                 (k_fac_diag_half, second)
//   T = L21 L11^-1                      (step 2)
//   X21 = -L22^-1 T                     (step 3)
// so that Li = [L11^-1 0; X21 L22^-1].  L21 is kept in Li's lower-left
// quadrant until X21 replaces it; S and then T live in the upper-right
// quadrant, which step 3 clears at the end.  Every launch takes the level's
// interior table unchanged: the half factorisations run one work-group per
// interior, the link products one per 64 x 64 macro tile (step 3: one per
// column of macro tiles, the only reader of that column of T).
constexpr int kHalf = 128;

template <typename C, typename In, bool SECOND, int W, typename Tab>
__global__ __launch_bounds__(64 * (W + 1))
__attribute__((amdgpu_waves_per_eu(W <= 3 ? 2 : 1))) void k_fac_diag_half(Tab tab)
{
    using T = typename Stor<C>::type;
    __shared__ CholSmem<T, 8> sm;
    const int64_t u = blockIdx.x;
    if (u >= tab.total) return;
    int64_t e;
    const auto& s = tab.get(u, e);
    const int np = s.np;
    const int64_t nn = (int64_t)np * np;
    const int64_t i = 2 * e + 1;
    T* Li = s.Li + e * nn;
    int bad;
    if constexpr (!SECOND)
        bad = chol_inv_block<C, 8, W, In>(s.Ad + i * nn, Li, kHalf, np, np, sm);
    else
        bad = chol_inv_block<C, 8, W, T>(Li + kHalf, Li + (int64_t)kHalf * np + kHalf, kHalf, np, np, sm);
    if (bad >= 0 && threadIdx.x == 0)
        report_notspd(s.info, s.level, (int)i, (int)(i << s.level), bad + (SECOND ? kHalf : 0));
}

template <typename C, typename In, int STEP, typename Tab>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_fac_diag_link(Tab tab)
{
    using T = typename Stor<C>::type;
    using Acc = typename AccT<C>::type;
    constexpr int MT = 64, KC = 16, R = MT / 32, H = kHalf, TP = H / MT;
    // work-groups per interior: one per macro tile, or (step 3) one per column of
    // macro tiles, so that each column of T has a single reader, which clears it
    constexpr int PER = STEP == 3 ? TP : TP * TP;
    __shared__ GemmSmem<T, MT, KC> sm;
    const int64_t w = xcd_local_index(blockIdx.x, gridDim.x);
    const int64_t u = w / PER;
    const int part = (int)(w % PER);
    if (u >= tab.total) return;
    int64_t e;
    const auto& s = tab.get(u, e);
    const int np = s.np;
    const int64_t nn = (int64_t)np * np;
    const int64_t i = 2 * e + 1;
    const In* A = s.Ad + i * nn;
    T* Li = s.Li + e * nn;
    T* L11i = Li;                          // L11^-1
    T* Low = Li + (int64_t)H * np;         // L21, then X21
    T* Scr = Li + H;                       // S, then T
    T* L22i = Li + (int64_t)H * np + H;    // L22^-1
    for (int q = 0; q < (STEP == 3 ? TP : 1); ++q) {
        const int tm = STEP == 3 ? q : part / TP, tn = STEP == 3 ? part : part % TP;
        if (STEP == 1 && tn > tm) return;  // S: lower macro tiles
        const int m0 = MT * tm, n0 = MT * tn;
        Acc acc[R][R];
        acc_zero<C, R, R>(acc);
        if constexpr (STEP == 0) {
            // L21 = A21 L11^-T; L11^-T is upper triangular, so k < n0 + MT
            const Term<In, T> terms[1] = {{{A + (int64_t)H * np, np, true}, {L11i, np, true}, 0, min(H, n0 + MT)}};
            wg_tile_product<C, MT, KC, 1, SKIP_TRI_B>(acc, terms, m0, n0, sm);
            wg_tile_foreach<C, MT>(acc, m0, n0, [&](int m, int n, T v) { Low[(int64_t)m * np + n] = v; });
        } else if constexpr (STEP == 1) {
            // S = A22 - L21 L21^T, lower triangle
            const bool sym = tm == tn;
            const Term<T, T> terms[1] = {{{Low, np, true}, {Low, np, true}, 0, H}};
            wg_tile_product<C, MT, KC, 1, SKIP_SYM>(acc, terms, m0, n0, sm, sym);
            const In* a22 = A + (int64_t)H * np + H;
            wg_tile_foreach<C, MT>(acc, m0, n0, [&](int m, int n, T v) {
                if (!sym || n <= m) Scr[(int64_t)m * np + n] = (T)a22[(int64_t)m * np + n] - v;
            });
        } else if constexpr (STEP == 2) {
            // T = L21 L11^-1; L11^-1 is lower triangular, so k >= n0
            const Term<T, T> terms[1] = {{{Low, np, true}, {L11i, np, false}, n0, H}};
            wg_tile_product<C, MT, KC, 1>(acc, terms, m0, n0, sm);
            wg_tile_foreach<C, MT>(acc, m0, n0, [&](int m, int n, T v) { Scr[(int64_t)m * np + n] = v; });
        } else {
            // X21 = -L22^-1 T; L22^-1 is lower triangular, so k < m0 + MT
            const Term<T, T> terms[1] = {{{L22i, np, true}, {Scr, np, false}, 0, min(H, m0 + MT)}};
            wg_tile_product<C, MT, KC, 1>(acc, terms, m0, n0, sm);
            wg_tile_foreach<C, MT>(acc, m0, n0, [&](int m, int n, T v) { Low[(int64_t)m * np + n] = -v; });
        }
        __syncthreads();  // the LDS buffers are reused by the next tile
    }
    if constexpr (STEP == 3) {
        // this work-group was the only reader of column block `part` of T: clear it
        const int n0 = MT * part;
        for (int q = threadIdx.x; q < H * MT; q += blockDim.x)
            Scr[(int64_t)(q / MT) * np + n0 + q % MT] = (T)0;
    }
}

template <typename C, typename In, int R, int U, typename Tab>
__global__ __launch_bounds__(256) void k_fac_couple(Tab tab)
{
    using T = typename Stor<C>::type;
    using A = typename AccT<C>::type;
    const int64_t u = (int64_t)blockIdx.x * 4 + wave_id();
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, tp = np / (16 * R);
    const int64_t nn = (int64_t)np * np;
    const int64_t e = loc / (2 * tp * tp);
    const int rem = (int)(loc % (2 * tp * tp));
    const int which = rem / (tp * tp), t = rem % (tp * tp);
    const int m0 = 16 * R * (t / tp), n0 = 16 * R * (t % tp);
    const int64_t i = 2 * e + 1;
    const T* Li = s.Li + e * nn;
    A acc[R][R];
    acc_zero<C, R, R>(acc);
    if (which == 0) {
        // Wt = A[i,i-1]^T Li^T; Li^T upper: k < n0 + 16R
        wave_mma<C, R, R, false, true, false, U>(acc, s.As + (i - 1) * nn + m0, np, Li + (int64_t)n0 * np, np, 0,
                                                 0, 0, min(np, n0 + 16 * R));
        T* out = s.Wt + e * nn;
        acc_foreach<C, R, R>(acc, m0, n0, [&](int m, int n, T v) { out[(int64_t)m * np + n] = v; });
    } else {
        if (i + 1 >= s.M) return;
        // Pr = A[i+1,i] * Li^T; Li^T upper: k < n0 + 16R
        wave_mma<C, R, R, true, true, false, U>(acc, s.As + i * nn + (int64_t)m0 * np, np, Li + (int64_t)n0 * np,
                                                np, 0, 0, 0, min(np, n0 + 16 * R));
        T* out = s.Pr + e * nn;
        acc_foreach<C, R, R>(acc, m0, n0, [&](int m, int n, T v) { out[(int64_t)m * np + n] = v; });
    }
}

template <typename C, typename In, int R, int U, typename Tab>
__global__ __launch_bounds__(256) void k_fac_schur(Tab tab)
{
    using T = typename Stor<C>::type;
    using A = typename AccT<C>::type;
    const int64_t u = (int64_t)blockIdx.x * 4 + wave_id();
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, tp = np / (16 * R);
    const int64_t nn = (int64_t)np * np;
    const int tl = tp * (tp + 1) / 2;
    const int per = tl + tp * tp;
    const int64_t j = loc / per;
    const int rem = (int)(loc % per);
    const int Mn = (s.M + 1) / 2;
    A acc[R][R];
    acc_zero<C, R, R>(acc);
    if (rem < tl) {
        int tm = 0;
        while ((tm + 1) * (tm + 2) / 2 <= rem) ++tm;
        const int tn = rem - tm * (tm + 1) / 2;
        const int m0 = 16 * R * tm, n0 = 16 * R * tn;
        if (j >= 1) {
            const T* P = s.Pr + (j - 1) * nn;
            wave_mma<C, R, R, true, true, false, U>(acc, P + (int64_t)m0 * np, np, P + (int64_t)n0 * np, np, 0, 0, 0,
                                                    np);
        }
        if (2 * j + 1 < s.M) {
            const T* W = s.Wt + j * nn;
            wave_mma<C, R, R, true, true, false, U>(acc, W + (int64_t)m0 * np, np, W + (int64_t)n0 * np, np, 0, 0, 0,
                                                    np);
        }
        const In* a = s.Ad + 2 * j * nn;
        T* out = s.Adn + j * nn;
        acc_foreach<C, R, R>(acc, m0, n0, [&](int m, int n, T v) {
            out[(int64_t)m * np + n] = (T)a[(int64_t)m * np + n] - v;
        });
    } else {
        if (j >= Mn - 1) return;
        const int t = rem - tl;
        const int m0 = 16 * R * (t / tp), n0 = 16 * R * (t % tp);
        const T* P = s.Pr + j * nn;
        const T* W = s.Wt + j * nn;
        wave_mma<C, R, R, true, true, false, U>(acc, P + (int64_t)m0 * np, np, W + (int64_t)n0 * np, np, 0, 0, 0,
                                                np);
        T* out = s.Asn + j * nn;
        acc_foreach<C, R, R>(acc, m0, n0, [&](int m, int n, T v) { out[(int64_t)m * np + n] = -v; });
    }
}

// Work-group versions of k_fac_couple / k_fac_schur for block sizes that are
// a multiple of the macro tile MT (see bds_gemm.hpp).
//   couple: unit = (interior e, product in {Wt, Pr}, macro tile)
//   schur:  unit = (separator j, tile): the lower macro tiles of S_jj, then the
//           macro tiles of S_{j+1,j} (none for the last separator), so that the
//           work-groups reading Wt[j] and Pr[j] run side by side
static int64_t units_fac_couple_wg(int M, int np, int MT)
{
    const int tp = np / MT;
    return (int64_t)(M / 2) * 2 * tp * tp;
}
static int64_t units_fac_schur_wg(int M, int np, int MT)
{
    const int tp = np / MT;
    return (int64_t)((M + 1) / 2) * (tp * (tp + 1) / 2 + tp * tp);
}

template <typename C, typename In, int MT, int KC, typename Tab>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MT <= 64 ? 4 : 2))) void k_fac_couple_wg(Tab tab)
{
    using T = typename Stor<C>::type;
    using Acc = typename AccT<C>::type;
    constexpr int R = MT / 32;
    __shared__ GemmSmem<T, MT, KC> sm;
    const int64_t u = xcd_local_index(blockIdx.x, gridDim.x);
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, tp = np / MT;
    const int64_t nn = (int64_t)np * np;
    const int64_t e = loc / (2 * tp * tp);
    const int rem = (int)(loc % (2 * tp * tp));
    const int which = rem / (tp * tp), t = rem % (tp * tp);
    const int m0 = MT * (t / tp), n0 = MT * (t % tp);
    const int64_t i = 2 * e + 1;
    if (which == 1 && i + 1 >= s.M) return;
    Acc acc[R][R];
    acc_zero<C, R, R>(acc);
    // Wt = A[i,i-1]^T Li^T, Pr = A[i+1,i] Li^T; Li^T is upper triangular, so k < n0 + MT
    const View<In> op = which == 0 ? View<In>{s.As + (i - 1) * nn, np, false} : View<In>{s.As + i * nn, np, true};
    const Term<In, T> terms[1] = {{op, {s.Li + e * nn, np, true}, 0, min(np, n0 + MT)}};
    wg_tile_product<C, MT, KC, 1, SKIP_TRI_B>(acc, terms, m0, n0, sm);
    T* out = (which == 0 ? s.Wt : s.Pr) + e * nn;
    wg_tile_foreach<C, MT>(acc, m0, n0, [&](int m, int n, T v) { out[(int64_t)m * np + n] = v; });
}

template <typename C, typename In, int MT, int KC, typename Tab>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MT <= 64 ? 4 : 2))) void k_fac_schur_wg(Tab tab)
{
    using T = typename Stor<C>::type;
    using Acc = typename AccT<C>::type;
    constexpr int R = MT / 32;
    __shared__ GemmSmem<T, MT, KC> sm;
    const int64_t u = xcd_local_index(blockIdx.x, gridDim.x);
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, tp = np / MT;
    const int64_t nn = (int64_t)np * np;
    const int tl = tp * (tp + 1) / 2;
    const int64_t j = loc / (tl + tp * tp);
    const int rem = (int)(loc % (tl + tp * tp));
    const bool diag = rem < tl;
    if (!diag && j >= (s.M + 1) / 2 - 1) return;
    int m0, n0;
    if (diag) {
        int tm = 0;
        while ((tm + 1) * (tm + 2) / 2 <= rem) ++tm;
        m0 = MT * tm;
        n0 = MT * (rem - tm * (tm + 1) / 2);
    } else {
        m0 = MT * ((rem - tl) / tp);
        n0 = MT * ((rem - tl) % tp);
    }
    // off-diagonal: S_{j+1,j} = -Pr(j) Wt(j)^T
    // diagonal: S_jj = A_jj - Pr(j-1) Pr(j-1)^T - Wt(j) Wt(j)^T; a term absent at
    // either end of the chain gets no chunks (its pointers are not read)
    View<T> a0{s.Pr + j * nn, np, true}, b0{s.Wt + j * nn, np, true};
    const View<T> w{s.Wt + j * nn, np, true};
    int k0end = np, k1end = 0;
    if (diag) {
        const bool left = j >= 1;
        a0.p = b0.p = left ? s.Pr + (j - 1) * nn : s.Pr;
        k0end = left ? np : 0;
        k1end = 2 * j + 1 < s.M ? np : 0;
    }
    const Term<T, T> terms[2] = {{a0, b0, 0, k0end}, {w, w, 0, k1end}};
    Acc acc[R][R];
    acc_zero<C, R, R>(acc);
    // only the lower triangle of S_jj is kept (every reader of a diagonal block
    // reads its lower triangle): diagonal macro tiles skip their strictly upper
    // 16 x 16 tiles and store no element above the diagonal
    const bool sym = diag && m0 == n0;
    wg_tile_product<C, MT, KC, 2, SKIP_SYM>(acc, terms, m0, n0, sm, sym);
    if (diag) {
        const In* a = s.Ad + 2 * j * nn;
        T* out = s.Adn + j * nn;
        wg_tile_foreach<C, MT>(acc, m0, n0, [&](int m, int n, T v) {
            if (!sym || n <= m) out[(int64_t)m * np + n] = (T)a[(int64_t)m * np + n] - v;
        });
    } else {
        T* out = s.Asn + j * nn;
        wg_tile_foreach<C, MT>(acc, m0, n0, [&](int m, int n, T v) { out[(int64_t)m * np + n] = -v; });
    }
}

// Coarse system: C_i = A_ii - Lsc[i-1] Lsc[i-1]^T, Lc[i] = chol(C_i)^-1,
// Lsc[i] = A_{i+1,i} Lc[i]^T.  One work-group per system.
template <typename In, int NT, int R, typename Tab>
__global__ __launch_bounds__(chol_threads<NT>()) void k_coarse_factor(Tab tab)
{
    using A = typename AccT<double>::type;
    constexpr int W = CholWaves<NT>::value;
    constexpr int WB = W + 1;  // waves in the block
    __shared__ CholSmem<double, NT> sm;
    const int64_t u = blockIdx.x;
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, tp = np / (16 * R), w = wave_id();
    const int64_t nn = (int64_t)np * np;
    for (int i = 0; i < s.Mc; ++i) {
        const In* a = s.Ad + i * nn;
        for (int t = w; t < tp * tp; t += WB) {
            const int m0 = 16 * R * (t / tp), n0 = 16 * R * (t % tp);
            A acc[R][R];
            acc_zero<double, R, R>(acc);
            if (i > 0) {
                const double* P = s.Lsc + (int64_t)(i - 1) * nn;
                wave_mma<double, R, R, true, true>(acc, P + (int64_t)m0 * np, np, P + (int64_t)n0 * np, np, 0,
                                                   0, 0, np);
            }
            acc_foreach<double, R, R>(acc, m0, n0, [&](int m, int n, double v) {
                s.Cw[(int64_t)m * np + n] = (double)a[(int64_t)m * np + n] - v;
            });
        }
        __syncthreads();
        double* Lci = s.Lc + (int64_t)i * nn;
        const int bad = chol_inv_block<double, NT, W, double>(s.Cw, Lci, np, np, np, sm);
        if (bad >= 0 && threadIdx.x == 0)
            report_notspd(s.info, s.level, i, i << s.level, bad);
        if (i + 1 < s.Mc) {
            const In* c = s.As + (int64_t)i * nn;
            for (int t = w; t < tp * tp; t += WB) {
                const int m0 = 16 * R * (t / tp), n0 = 16 * R * (t % tp);
                A acc[R][R];
                acc_zero<double, R, R>(acc);
                wave_mma<double, R, R, true, true>(acc, c + (int64_t)m0 * np, np, Lci + (int64_t)n0 * np, np, 0,
                                                   0, 0, min(np, n0 + 16 * R));
                double* out = s.Lsc + (int64_t)i * nn;
                acc_foreach<double, R, R>(acc, m0, n0,
                                          [&](int m, int n, double v) { out[(int64_t)m * np + n] = v; });
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// solve (vectors in FP64; factor blocks of type T converted on load)

template <typename T, int R, int U, typename Tab>
__global__ __launch_bounds__(256) void k_sol_fwd_int(Tab tab)
{
    using A = typename AccT<double>::type;
    const int64_t u = (int64_t)blockIdx.x * 4 + wave_id();
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, d = s.d, tp = np / (16 * R), dc = (d + 15) / 16;
    const int64_t nn = (int64_t)np * np, nd = (int64_t)np * d;
    const int64_t e = loc / (tp * dc);
    const int rem = (int)(loc % (tp * dc));
    const int m0 = 16 * R * (rem / dc), c0 = 16 * (rem % dc);
    const int64_t i = 2 * e + 1;
    A acc[R][1];
    acc_zero<double, R, 1>(acc);
    wave_mma<double, R, 1, true, false, true, U>(acc, s.Li + e * nn + (int64_t)m0 * np, np, s.B + i * nd + c0, d,
                                                 0, 0, 0, min(np, m0 + 16 * R), d - c0);
    double* y = s.Y + e * nd;
    acc_foreach<double, R, 1>(acc, m0, c0, [&](int m, int n, double v) {
        if (n < d) y[(int64_t)m * d + n] = v;
    });
}

template <typename T, int R, int U, typename Tab>
__global__ __launch_bounds__(256) void k_sol_fwd_sep(Tab tab)
{
    using A = typename AccT<double>::type;
    const int64_t u = (int64_t)blockIdx.x * 4 + wave_id();
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, d = s.d, tp = np / (16 * R), dc = (d + 15) / 16;
    const int64_t nn = (int64_t)np * np, nd = (int64_t)np * d;
    const int64_t j = loc / (tp * dc);
    const int rem = (int)(loc % (tp * dc));
    const int m0 = 16 * R * (rem / dc), c0 = 16 * (rem % dc);
    A acc[R][1];
    acc_zero<double, R, 1>(acc);
    if (j >= 1)
        wave_mma<double, R, 1, true, false, true, U>(acc, s.Pr + (j - 1) * nn + (int64_t)m0 * np, np,
                                                     s.Y + (j - 1) * nd + c0, d, 0, 0, 0, np, d - c0);
    if (2 * j + 1 < s.M)
        wave_mma<double, R, 1, true, false, true, U>(acc, s.Wt + j * nn + (int64_t)m0 * np, np,
                                                     s.Y + j * nd + c0, d, 0, 0, 0, np, d - c0);
    const double* b = s.B + 2 * j * nd;
    double* out = s.Bn + j * nd;
    acc_foreach<double, R, 1>(acc, m0, c0, [&](int m, int n, double v) {
        if (n < d) out[(int64_t)m * d + n] = b[(int64_t)m * d + n] - v;
    });
}

// One work-group of min(4, np / 16R) waves per (interior, 16 columns); for
// launches of at most one work-group per CU, the unrolled form with up to 4
// waves (U = 4) or, where a block has more row tiles, 8 waves with two k-steps
// in flight (U = 2, which fits the 256 registers per lane of 8 waves); the
// launch provides np * 16 doubles of dynamic LDS for the corrected right-hand side.
template <typename T, int R, int U, typename Tab>
__global__ __launch_bounds__(U == 2 ? 512 : 256) void k_sol_bwd(Tab tab)
{
    using A = typename AccT<double>::type;
    extern __shared__ double tsm[];
    const int64_t u = blockIdx.x;
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, d = s.d, tp = np / (16 * R), dc = (d + 15) / 16, w = wave_id();
    const int nw = blockDim.x >> 6;
    const int64_t nn = (int64_t)np * np, nd = (int64_t)np * d;
    const int64_t e = loc / dc;
    const int c0 = 16 * (int)(loc % dc);
    const int64_t i = 2 * e + 1;
    const int Mn = (s.M + 1) / 2;
    for (int t = w; t < tp; t += nw) {
        const int m0 = 16 * R * t;
        A acc[R][1];
        acc_zero<double, R, 1>(acc);
        wave_mma<double, R, 1, false, false, true, U>(acc, s.Wt + e * nn + m0, np, s.Xn + e * nd + c0, d, 0, 0,
                                                      0, np, d - c0);
        if (i + 1 < s.M)
            wave_mma<double, R, 1, false, false, true, U>(acc, s.Pr + e * nn + m0, np, s.Xn + (e + 1) * nd + c0,
                                                          d, 0, 0, 0, np, d - c0);
        const double* y = s.Y + e * nd;
        acc_foreach<double, R, 1>(acc, m0, 0, [&](int m, int n, double v) {
            tsm[m * 16 + n] = (c0 + n < d) ? y[(int64_t)m * d + c0 + n] - v : 0.0;
        });
    }
    __syncthreads();
    for (int t = w; t < tp; t += nw) {
        const int m0 = 16 * R * t;
        A acc[R][1];
        acc_zero<double, R, 1>(acc);
        // Li^T is upper triangular: k >= m0
        wave_mma<double, R, 1, false, false, false, U>(acc, s.Li + e * nn + m0, np, tsm, 16, 0, 0, m0, np);
        double* x = s.X + i * nd;
        acc_foreach<double, R, 1>(acc, m0, c0, [&](int m, int n, double v) {
            if (n < d) x[(int64_t)m * d + n] = v;
        });
    }
    // separators: X[2e] = Xn[e]; the last separator of an odd level too
    const int cw = min(16, d - c0);
    for (int q = threadIdx.x; q < np * cw; q += blockDim.x) {
        const int r = q / cw, c = c0 + q % cw;
        s.X[2 * e * nd + (int64_t)r * d + c] = s.Xn[e * nd + (int64_t)r * d + c];
        if ((s.M & 1) && e == s.M / 2 - 1)
            s.X[(int64_t)(s.M - 1) * nd + (int64_t)r * d + c] = s.Xn[(int64_t)(Mn - 1) * nd + (int64_t)r * d + c];
    }
}

// Coarse block forward/backward substitution, one work-group per (system, 16 columns).
template <int R, typename Tab>
__global__ __launch_bounds__(256) void k_coarse_solve(Tab tab)
{
    using A = typename AccT<double>::type;
    __shared__ double tsm[kMaxNP * 16];
    const int64_t u = blockIdx.x;
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, d = s.d, tp = np / (16 * R), w = wave_id();
    const int64_t nn = (int64_t)np * np, nd = (int64_t)np * d;
    const int c0 = 16 * (int)loc;
    for (int i = 0; i < s.Mc; ++i) {
        for (int t = w; t < tp; t += 4) {
            const int m0 = 16 * R * t;
            A acc[R][1];
            acc_zero<double, R, 1>(acc);
            if (i > 0)
                wave_mma<double, R, 1, true, false, true>(acc, s.Lsc + (int64_t)(i - 1) * nn + (int64_t)m0 * np,
                                                          np, s.Y + (int64_t)(i - 1) * nd + c0, d, 0, 0, 0, np,
                                                          d - c0);
            const double* b = s.B + (int64_t)i * nd;
            acc_foreach<double, R, 1>(acc, m0, 0, [&](int m, int n, double v) {
                tsm[m * 16 + n] = (c0 + n < d) ? b[(int64_t)m * d + c0 + n] - v : 0.0;
            });
        }
        __syncthreads();
        for (int t = w; t < tp; t += 4) {
            const int m0 = 16 * R * t;
            A acc[R][1];
            acc_zero<double, R, 1>(acc);
            wave_mma<double, R, 1, true, false>(acc, s.Lc + (int64_t)i * nn + (int64_t)m0 * np, np, tsm, 16, 0,
                                                0, 0, min(np, m0 + 16 * R));
            double* y = s.Y + (int64_t)i * nd;
            acc_foreach<double, R, 1>(acc, m0, c0, [&](int m, int n, double v) {
                if (n < d) y[(int64_t)m * d + n] = v;
            });
        }
        __syncthreads();
    }
    for (int i = s.Mc - 1; i >= 0; --i) {
        for (int t = w; t < tp; t += 4) {
            const int m0 = 16 * R * t;
            A acc[R][1];
            acc_zero<double, R, 1>(acc);
            if (i + 1 < s.Mc)
                wave_mma<double, R, 1, false, false, true>(acc, s.Lsc + (int64_t)i * nn + m0, np,
                                                           s.X + (int64_t)(i + 1) * nd + c0, d, 0, 0, 0, np,
                                                           d - c0);
            const double* y = s.Y + (int64_t)i * nd;
            acc_foreach<double, R, 1>(acc, m0, 0, [&](int m, int n, double v) {
                tsm[m * 16 + n] = (c0 + n < d) ? y[(int64_t)m * d + c0 + n] - v : 0.0;
            });
        }
        __syncthreads();
        for (int t = w; t < tp; t += 4) {
            const int m0 = 16 * R * t;
            A acc[R][1];
            acc_zero<double, R, 1>(acc);
            wave_mma<double, R, 1, false, false>(acc, s.Lc + (int64_t)i * nn + m0, np, tsm, 16, 0, 0, m0, np);
            double* x = s.X + (int64_t)i * nd;
            acc_foreach<double, R, 1>(acc, m0, c0, [&](int m, int n, double v) {
                if (n < d) x[(int64_t)m * d + n] = v;
            });
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// refinement: residual, update and norms (FP64)

// R_i = B_i - sym(A_ii) X_i - A_{i,i-1} X_{i-1} - A_{i+1,i}^T X_{i+1}
template <int R, typename Tab>
__global__ __launch_bounds__(256) void k_residual(Tab tab)
{
    using A = typename AccT<double>::type;
    // consecutive block rows on one XCD: rows i and i + 1 both read A_{i+1,i},
    // and the second read then comes from that XCD's L2 instead of HBM
    const int64_t u = xcd_local_index(blockIdx.x, gridDim.x) * 4 + wave_id();
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    const int np = s.np, d = s.d, tp = np / (16 * R), dc = (d + 15) / 16;
    const int64_t nn = (int64_t)np * np, nd = (int64_t)np * d;
    const int64_t i = loc / (tp * dc);
    const int rem = (int)(loc % (tp * dc));
    const int m0 = 16 * R * (rem / dc), c0 = 16 * (rem % dc);
    const int l = lane_id(), li = l & 15, g = l >> 4;
    A acc[R][1];
    acc_zero<double, R, 1>(acc);
    {
        // diagonal block, symmetric completion of its lower triangle
        const double* a = s.Ad + i * nn;
        const double* x = s.X + i * nd + c0;
        const bool ok = c0 + li < d;
        for (int kc = 0; kc < np; kc += 16) {
            const int k = kc + 4 * g;
            double av[R][4], bv[4];
#pragma unroll
            for (int ta = 0; ta < R; ++ta) {
                const int m = m0 + 16 * ta + li;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    av[ta][q] = (m >= k + q) ? a[(int64_t)m * np + k + q] : a[(int64_t)(k + q) * np + m];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) bv[q] = ok ? x[(int64_t)(k + q) * d + li] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int ta = 0; ta < R; ++ta) acc[ta][0] = mma(av[ta][q], bv[q], acc[ta][0]);
        }
    }
    if (i > 0)
        wave_mma<double, R, 1, true, false, true>(acc, s.As + (i - 1) * nn + (int64_t)m0 * np, np,
                                                  s.X + (i - 1) * nd + c0, d, 0, 0, 0, np, d - c0);
    if (i + 1 < s.N)
        wave_mma<double, R, 1, false, false, true>(acc, s.As + i * nn + m0, np, s.X + (i + 1) * nd + c0, d, 0,
                                                   0, 0, np, d - c0);
    const double* b = s.B + i * nd;
    double* r = s.R + i * nd;
    acc_foreach<double, R, 1>(acc, m0, c0, [&](int m, int n, double v) {
        if (n < d) r[(int64_t)m * d + n] = b[(int64_t)m * d + n] - v;
    });
}

// X += C per block with per-block partial sums of C^2 and X^2, then one
// work-group per record sums the partials in a fixed order.
template <typename Tab>
__global__ __launch_bounds__(256) void k_axpy_norm(Tab tab)
{
    __shared__ double red[2][256];
    const int64_t u = blockIdx.x;
    if (u >= tab.total) return;
    int64_t i;
    const auto& s = tab.get(u, i);
    const int64_t nd = (int64_t)s.np * s.d;
    double sc = 0, sx = 0;
    for (int64_t q = threadIdx.x; q < nd; q += blockDim.x) {
        const double c = s.C[i * nd + q];
        const double x = s.X[i * nd + q] + c;
        s.X[i * nd + q] = x;
        sc += c * c;
        sx += x * x;
    }
    red[0][threadIdx.x] = sc;
    red[1][threadIdx.x] = sx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        s.part[2 * i] = red[0][0];
        s.part[2 * i + 1] = red[1][0];
    }
}

template <typename Tab>
__global__ __launch_bounds__(256) void k_norm_final(Tab tab)
{
    __shared__ double red[2][256];
    const int64_t u = blockIdx.x;
    if (u >= tab.total) return;
    int64_t loc;
    const auto& s = tab.get(u, loc);
    double sc = 0, sx = 0;
    for (int64_t q = threadIdx.x; q < s.N; q += blockDim.x) {
        sc += s.part[2 * q];
        sx += s.part[2 * q + 1];
    }
    red[0][threadIdx.x] = sc;
    red[1][threadIdx.x] = sx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        s.out[0] = red[0][0];
        s.out[1] = red[1][0];
    }
}

// ---------------------------------------------------------------------------
// adjoint: dAd[i] = -(G_i X_i^T + X_i G_i^T)/2, dAs[i] = -(G_{i+1} X_i^T + X_{i+1} G_i^T)

__global__ __launch_bounds__(256) void k_adjoint(AdjArgs a)
{
    const int64_t blk = blockIdx.x;  // 0..N-1: diagonal, N..2N-2: coupling
    const int n = a.n, np = a.np, d = a.d;
    const int64_t nd = (int64_t)np * d;
    const bool diag = blk < a.N;
    const int64_t i = diag ? blk : blk - a.N;
    const double* G0 = a.G + i * nd;
    const double* X0 = a.X + i * nd;
    const double* G1 = diag ? G0 : a.G + (i + 1) * nd;
    const double* X1 = diag ? X0 : a.X + (i + 1) * nd;
    double* out = diag ? a.dAd + i * (int64_t)n * n : a.dAs + i * (int64_t)n * n;
    const double scale = diag ? -0.5 : -1.0;
    for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
        const int r = q / n, c = q % n;
        double t = 0;
        for (int k = 0; k < d; ++k)
            t += G1[(int64_t)r * d + k] * X0[(int64_t)c * d + k] + X1[(int64_t)r * d + k] * G0[(int64_t)c * d + k];
        out[q] = scale * t;
    }
}

// ---------------------------------------------------------------------------
// packing for n not a multiple of 16

__global__ void k_pack_blocks(const double* src, double* dst, int64_t nblk, int n, int np, int diag)
{
    const int64_t total = nblk * np * np;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = q / ((int64_t)np * np);
        const int r = (int)((q / np) % np), c = (int)(q % np);
        double v;
        if (r < n && c < n)
            v = src[b * n * n + (int64_t)r * n + c];
        else
            v = (diag && r == c) ? 1.0 : 0.0;
        dst[q] = v;
    }
}

__global__ void k_pack_rhs(const double* src, double* dst, int64_t nblk, int n, int np, int d)
{
    const int64_t total = nblk * np * d;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = q / ((int64_t)np * d);
        const int r = (int)((q / d) % np), c = (int)(q % d);
        dst[q] = r < n ? src[(b * n + r) * d + c] : 0.0;
    }
}

__global__ void k_unpack_rhs(const double* src, double* dst, int64_t nblk, int n, int np, int d)
{
    const int64_t total = nblk * n * d;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = q / ((int64_t)n * d);
        const int r = (int)((q / d) % n), c = (int)(q % d);
        dst[q] = src[(b * np + r) * d + c];
    }
}

// Table-driven packing for batched systems: one work-group per block.
template <typename Tab>
__global__ __launch_bounds__(256) void k_pack_tab(Tab tab)
{
    const int64_t u = blockIdx.x;
    if (u >= tab.total) return;
    int64_t b;
    const auto& s = tab.get(u, b);
    const int n = s.n, np = s.np, c = s.cols;
    if (s.mode == PACK_UNPACK_RHS) {
        const double* src = s.src + b * (int64_t)np * c;
        double* dst = s.dst + b * (int64_t)n * c;
        for (int q = threadIdx.x; q < n * c; q += blockDim.x) dst[q] = src[(q / c) * c + q % c];
        return;
    }
    const int sc = (s.mode == PACK_RHS) ? c : n;     // source columns
    const int dc = (s.mode == PACK_RHS) ? c : np;    // destination columns
    const int dr = np;
    const double* src = s.src + b * (int64_t)n * sc;
    double* dst = s.dst + b * (int64_t)dr * dc;
    for (int q = threadIdx.x; q < dr * dc; q += blockDim.x) {
        const int r = q / dc, cc = q % dc;
        double v;
        if (r < n && cc < sc)
            v = src[(int64_t)r * sc + cc];
        else
            v = (s.mode == PACK_DIAG && r == cc) ? 1.0 : 0.0;
        dst[q] = v;
    }
}

// Per-record refinement outcome: ic[2k] = iterations, ic[2k+1] = converged.
__global__ void k_set_refine_info_tab(bds_info* info, const int* ic, int K)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    info[k].iters = ic[2 * k];
    info[k].converged = ic[2 * k + 1];
    if (!ic[2 * k + 1]) atomicCAS(&info[k].status, 0, (int)BDS_ENOCONV);
}

__global__ void k_clear_info(bds_info* info, int K)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < K) info[q] = bds_info{0, 0, 0, 0, 0, 0, 0, 0};
}

__global__ void k_set_refine_info(bds_info* info, int iters, int converged)
{
    if (threadIdx.x == 0) {
        info->iters = iters;
        info->converged = converged;
        if (!converged) atomicCAS(&info->status, 0, (int)BDS_ENOCONV);
    }
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned grid_waves(int64_t units) { return (unsigned)((units + 3) / 4); }

// Register-tile bound NT (np = 16 nt, nt <= NT) of the block factorisation kernels.
template <int NT> struct NtTag { static constexpr int value = NT; };
// Compute units of the current device (cached per device).
static int cu_count()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

Tiling level_tiling(const Tiling& tl, int32_t req, int M, int np)
{
    Tiling t = tl;
    const int64_t few = cu_count();
    if (!(req & 15) && t.couple >= BDS_TILE_G64 && units_fac_couple(M, np, t.couple) <= few) t.couple = BDS_TILE_W16;
    if (!((req >> 4) & 15) && t.schur >= BDS_TILE_G64 && units_fac_schur(M, np, t.schur) <= few)
        t.schur = BDS_TILE_W16;
    return t;
}

template <typename F> static hipError_t dispatch_nt(int np_max, F&& f)
{
    const int nt = np_max / 16;
    if (nt <= 2) return f(NtTag<2>{});
    if (nt <= 4) return f(NtTag<4>{});
    if (nt <= 8) return f(NtTag<8>{});
    return f(NtTag<16>{});
}

// Run `launch(table)` on the single record (tab == nullptr) or on the K
// records at tab with prefix sums start; the table's unit total is `total`.
template <typename Rec, typename F>
static hipError_t with_table(const Rec& one, const Rec* tab, const int64_t* start, int K, int64_t total, F&& launch)
{
    if (total <= 0) return hipSuccess;
    if (!tab) return launch(One<Rec>{one, total});
    return launch(Many<Rec>{tab, start, K, total});
}

template <typename C, typename In>
hipError_t launch_factor_level(const FacLv<typename Stor<C>::type, In>& one,
                               const FacLv<typename Stor<C>::type, In>* tab, const int64_t* sd,
                               const int64_t* sc, const int64_t* ss, int K, int64_t td, int64_t tc,
                               int64_t ts, int np, const Tiling& tl, hipStream_t st)
{
    hipError_t e = with_table(one, tab, sd, K, td, [&](auto t) {
        if (std::is_same<C, double>::value && np == 2 * kHalf) {
            // 2 x 2 recursion over 128-row halves (see k_fac_diag_half); FP64 only:
            // in FP32 the explicit 128-row inverses cost the refinement an
            // iteration at kappa ~ 1e6, which the 16-row pivot inverses do not
            // halves on levels with no more interiors than CUs: 16-wave work-groups (see k_fac_diag)
            const unsigned nb = (unsigned)td, ct = chol_threads<8>(), cw = 64 * (kWideWaves + 1);
            const bool wide = td <= cu_count();
            if (wide) BDS_TIMED("fac_diag", st, k_fac_diag_half<C, In, false, kWideWaves><<<nb, cw, 0, st>>>(t));
            else BDS_TIMED("fac_diag", st, k_fac_diag_half<C, In, false, CholWaves<8>::value><<<nb, ct, 0, st>>>(t));
            BDS_TIMED("fac_diag", st, k_fac_diag_link<C, In, 0><<<4 * nb, 256, 0, st>>>(t));
            BDS_TIMED("fac_diag", st, k_fac_diag_link<C, In, 1><<<4 * nb, 256, 0, st>>>(t));
            if (wide) BDS_TIMED("fac_diag", st, k_fac_diag_half<C, In, true, kWideWaves><<<nb, cw, 0, st>>>(t));
            else BDS_TIMED("fac_diag", st, k_fac_diag_half<C, In, true, CholWaves<8>::value><<<nb, ct, 0, st>>>(t));
            BDS_TIMED("fac_diag", st, k_fac_diag_link<C, In, 2><<<4 * nb, 256, 0, st>>>(t));
            BDS_TIMED("fac_diag", st, k_fac_diag_link<C, In, 3><<<2 * nb, 256, 0, st>>>(t));
            return hipGetLastError();
        }
        return dispatch_nt(np, [&](auto nt) {
            constexpr int NT = decltype(nt)::value;
            if constexpr (NT == 8) {
                if (td <= cu_count()) {
                    BDS_TIMED("fac_diag", st,
                              k_fac_diag<C, In, NT, kWideWaves><<<(unsigned)td, 64 * (kWideWaves + 1), 0, st>>>(t));
                    return hipGetLastError();
                }
            }
            BDS_TIMED("fac_diag", st,
                      k_fac_diag<C, In, NT, CholWaves<NT>::value><<<(unsigned)td, chol_threads<NT>(), 0, st>>>(t));
            return hipGetLastError();
        });
    });
    if (e != hipSuccess) return e;
    // chunk depth of the work-group products: 32 for FP32 products on blocks of 128
    // and more (measured faster there; 16 is faster for 64-wide blocks and BF16)
    const bool deep = std::is_same<C, float>::value && np >= 128;
    // per-wave tile products in launches of at most one work-group per CU: four
    // k-steps of loads in flight per wave (see launch_solve_fwd)
    const unsigned few = (unsigned)cu_count();
    e = with_table(one, tab, sc, K, tc, [&](auto t) {
        switch (tl.couple) {
        case BDS_TILE_G128:
            if (deep) BDS_TIMED("fac_couple", st, k_fac_couple_wg<C, In, 128, 32><<<(unsigned)tc, 256, 0, st>>>(t));
            else BDS_TIMED("fac_couple", st, k_fac_couple_wg<C, In, 128, 16><<<(unsigned)tc, 256, 0, st>>>(t));
            break;
        case BDS_TILE_G64:
            if (deep) BDS_TIMED("fac_couple", st, k_fac_couple_wg<C, In, 64, 32><<<(unsigned)tc, 256, 0, st>>>(t));
            else BDS_TIMED("fac_couple", st, k_fac_couple_wg<C, In, 64, 16><<<(unsigned)tc, 256, 0, st>>>(t));
            break;
        case BDS_TILE_W32:
            if (grid_waves(tc) <= few) BDS_TIMED("fac_couple", st, k_fac_couple<C, In, 2, 4><<<grid_waves(tc), 256, 0, st>>>(t));
            else BDS_TIMED("fac_couple", st, k_fac_couple<C, In, 2, 1><<<grid_waves(tc), 256, 0, st>>>(t));
            break;
        default:
            if (grid_waves(tc) <= few) BDS_TIMED("fac_couple", st, k_fac_couple<C, In, 1, 4><<<grid_waves(tc), 256, 0, st>>>(t));
            else BDS_TIMED("fac_couple", st, k_fac_couple<C, In, 1, 1><<<grid_waves(tc), 256, 0, st>>>(t));
            break;
        }
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return with_table(one, tab, ss, K, ts, [&](auto t) {
        switch (tl.schur) {
        case BDS_TILE_G128:
            if (deep) BDS_TIMED("fac_schur", st, k_fac_schur_wg<C, In, 128, 32><<<(unsigned)ts, 256, 0, st>>>(t));
            else BDS_TIMED("fac_schur", st, k_fac_schur_wg<C, In, 128, 16><<<(unsigned)ts, 256, 0, st>>>(t));
            break;
        case BDS_TILE_G64:
            if (deep) BDS_TIMED("fac_schur", st, k_fac_schur_wg<C, In, 64, 32><<<(unsigned)ts, 256, 0, st>>>(t));
            else BDS_TIMED("fac_schur", st, k_fac_schur_wg<C, In, 64, 16><<<(unsigned)ts, 256, 0, st>>>(t));
            break;
        case BDS_TILE_W32:
            if (grid_waves(ts) <= few) BDS_TIMED("fac_schur", st, k_fac_schur<C, In, 2, 4><<<grid_waves(ts), 256, 0, st>>>(t));
            else BDS_TIMED("fac_schur", st, k_fac_schur<C, In, 2, 1><<<grid_waves(ts), 256, 0, st>>>(t));
            break;
        default:
            if (grid_waves(ts) <= few) BDS_TIMED("fac_schur", st, k_fac_schur<C, In, 1, 4><<<grid_waves(ts), 256, 0, st>>>(t));
            else BDS_TIMED("fac_schur", st, k_fac_schur<C, In, 1, 1><<<grid_waves(ts), 256, 0, st>>>(t));
            break;
        }
        return hipGetLastError();
    });
}

template <typename In>
hipError_t launch_coarse_factor(const CoarseFac<In>& one, const CoarseFac<In>* tab, int K, int np_max,
                                hipStream_t st)
{
    if (!tab) {
        One<CoarseFac<In>> o{one, 1};
        return dispatch_nt(one.np, [&](auto nt) {
            constexpr int NT = decltype(nt)::value;
            if (one.np % 32 == 0)
                BDS_TIMED("coarse_factor", st, k_coarse_factor<In, NT, 2><<<1, chol_threads<NT>(), 0, st>>>(o));
            else
                BDS_TIMED("coarse_factor", st, k_coarse_factor<In, NT, 1><<<1, chol_threads<NT>(), 0, st>>>(o));
            return hipGetLastError();
        });
    }
    // one work-group per record
    if (K <= 0) return hipSuccess;
    Many<CoarseFac<In>> m{tab, nullptr, K, K};
    return dispatch_nt(np_max, [&](auto nt) {
        constexpr int NT = decltype(nt)::value;
        BDS_TIMED("coarse_factor", st, k_coarse_factor<In, NT, 1><<<(unsigned)K, chol_threads<NT>(), 0, st>>>(m));
        return hipGetLastError();
    });
}

// Solve launches with at most one work-group per CU cannot hide the latency
// of a wave's k-steps behind other waves: their kernels unroll the k loop
// (kSolveUnroll steps in flight per wave) instead.
constexpr int kSolveUnroll = 4;

template <typename T>
hipError_t launch_solve_fwd(const SolLv<T>& one, const SolLv<T>* tab, const int64_t* si, const int64_t* ss,
                            int K, int64_t ti, int64_t ts, int np, const Tiling& tl, hipStream_t st)
{
    const bool r2 = tl.sol == BDS_TILE_W32;
    hipError_t e = with_table(one, tab, si, K, ti, [&](auto t) {
        const unsigned g = grid_waves(ti);
        const bool few = g <= (unsigned)cu_count();
        if (r2 && few) BDS_TIMED("sol_fwd_int", st, k_sol_fwd_int<T, 2, kSolveUnroll><<<g, 256, 0, st>>>(t));
        else if (r2) BDS_TIMED("sol_fwd_int", st, k_sol_fwd_int<T, 2, 1><<<g, 256, 0, st>>>(t));
        else if (few) BDS_TIMED("sol_fwd_int", st, k_sol_fwd_int<T, 1, kSolveUnroll><<<g, 256, 0, st>>>(t));
        else BDS_TIMED("sol_fwd_int", st, k_sol_fwd_int<T, 1, 1><<<g, 256, 0, st>>>(t));
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return with_table(one, tab, ss, K, ts, [&](auto t) {
        const unsigned g = grid_waves(ts);
        const bool few = g <= (unsigned)cu_count();
        if (r2 && few) BDS_TIMED("sol_fwd_sep", st, k_sol_fwd_sep<T, 2, kSolveUnroll><<<g, 256, 0, st>>>(t));
        else if (r2) BDS_TIMED("sol_fwd_sep", st, k_sol_fwd_sep<T, 2, 1><<<g, 256, 0, st>>>(t));
        else if (few) BDS_TIMED("sol_fwd_sep", st, k_sol_fwd_sep<T, 1, kSolveUnroll><<<g, 256, 0, st>>>(t));
        else BDS_TIMED("sol_fwd_sep", st, k_sol_fwd_sep<T, 1, 1><<<g, 256, 0, st>>>(t));
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_solve_bwd(const SolLv<T>& one, const SolLv<T>* tab, const int64_t* sb, int K, int64_t tb,
                            int np, const Tiling& tl, hipStream_t st)
{
    // a work-group's four waves share the np / (16 R) row tiles of one interior:
    // 32-row tiles only where that still leaves a tile per wave
    const int R = (tl.sol == BDS_TILE_W32 && np >= 128) ? 2 : 1;
    const size_t lds = (size_t)np * 16 * sizeof(double);
    return with_table(one, tab, sb, K, tb, [&](auto t) {
        const bool few = tb <= cu_count();
        const bool eight = few && np / (16 * R) > 4;
        const unsigned threads = 64u * (unsigned)std::min(eight ? 8 : 4, np / (16 * R));
        const unsigned g = (unsigned)tb;
        if (R == 2 && eight) BDS_TIMED("sol_bwd", st, k_sol_bwd<T, 2, 2><<<g, threads, lds, st>>>(t));
        else if (R == 2 && few) BDS_TIMED("sol_bwd", st, k_sol_bwd<T, 2, kSolveUnroll><<<g, threads, lds, st>>>(t));
        else if (R == 2) BDS_TIMED("sol_bwd", st, k_sol_bwd<T, 2, 1><<<g, threads, lds, st>>>(t));
        else if (eight) BDS_TIMED("sol_bwd", st, k_sol_bwd<T, 1, 2><<<g, threads, lds, st>>>(t));
        else if (few) BDS_TIMED("sol_bwd", st, k_sol_bwd<T, 1, kSolveUnroll><<<g, threads, lds, st>>>(t));
        else BDS_TIMED("sol_bwd", st, k_sol_bwd<T, 1, 1><<<g, threads, lds, st>>>(t));
        return hipGetLastError();
    });
}

hipError_t launch_coarse_solve(const CoarseSol& one, const CoarseSol* tab, const int64_t* start, int K,
                               int64_t tot, hipStream_t st)
{
    if (tot <= 0) return hipSuccess;
    if (!tab) {
        One<CoarseSol> o{one, tot};
        if (one.np % 32 == 0) BDS_TIMED("coarse_solve", st, k_coarse_solve<2><<<(unsigned)tot, 256, 0, st>>>(o));
        else BDS_TIMED("coarse_solve", st, k_coarse_solve<1><<<(unsigned)tot, 256, 0, st>>>(o));
    } else {
        Many<CoarseSol> m{tab, start, K, tot};
        BDS_TIMED("coarse_solve", st, k_coarse_solve<1><<<(unsigned)tot, 256, 0, st>>>(m));
    }
    return hipGetLastError();
}

hipError_t launch_residual(const ResidArgs& one, const ResidArgs* tab, const int64_t* start, int K, int64_t tot,
                           int np, hipStream_t st)
{
    return with_table(one, tab, start, K, tot, [&](auto t) {
        if (tile_r(np) == 2) BDS_TIMED("residual", st, k_residual<2><<<grid_waves(tot), 256, 0, st>>>(t));
        else BDS_TIMED("residual", st, k_residual<1><<<grid_waves(tot), 256, 0, st>>>(t));
        return hipGetLastError();
    });
}

hipError_t launch_axpy_norm(const AxpyArgs& one, const AxpyArgs* tab, const int64_t* start, int K, int64_t tot,
                            hipStream_t st)
{
    if (!tab) {
        One<AxpyArgs> o{one, tot};
        BDS_TIMED("axpy_norm", st, k_axpy_norm<<<(unsigned)tot, 256, 0, st>>>(o));
        o.total = 1;
        BDS_TIMED("norm_final", st, k_norm_final<<<1, 256, 0, st>>>(o));
    } else {
        if (tot <= 0) return hipSuccess;
        Many<AxpyArgs> m{tab, start, K, tot};
        BDS_TIMED("axpy_norm", st, k_axpy_norm<<<(unsigned)tot, 256, 0, st>>>(m));
        Many<AxpyArgs> f{tab, nullptr, K, K};
        BDS_TIMED("norm_final", st, k_norm_final<<<(unsigned)K, 256, 0, st>>>(f));
    }
    return hipGetLastError();
}

hipError_t launch_adjoint(const AdjArgs& a, hipStream_t st)
{
    const unsigned nb = (unsigned)(2 * a.N - 1);
    BDS_TIMED("adjoint", st, k_adjoint<<<nb, 256, 0, st>>>(a));
    return hipGetLastError();
}

static inline unsigned grid_elems(int64_t total)
{
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_pack_blocks(const double* src, double* dst, int64_t nblk, int n, int np, bool diag,
                              hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    BDS_TIMED("pack_blocks", st, k_pack_blocks<<<grid_elems(nblk * np * np), 256, 0, st>>>(src, dst, nblk, n, np, diag ? 1 : 0));
    return hipGetLastError();
}

hipError_t launch_pack_rhs(const double* src, double* dst, int64_t nblk, int n, int np, int d, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    BDS_TIMED("pack_rhs", st, k_pack_rhs<<<grid_elems(nblk * np * d), 256, 0, st>>>(src, dst, nblk, n, np, d));
    return hipGetLastError();
}

hipError_t launch_unpack_rhs(const double* src, double* dst, int64_t nblk, int n, int np, int d, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    BDS_TIMED("unpack_rhs", st, k_unpack_rhs<<<grid_elems(nblk * n * d), 256, 0, st>>>(src, dst, nblk, n, np, d));
    return hipGetLastError();
}

hipError_t launch_pack_tab(const PackRec* tab, const int64_t* start, int K, int64_t tot, hipStream_t st)
{
    if (tot <= 0) return hipSuccess;
    Many<PackRec> m{tab, start, K, tot};
    BDS_TIMED("pack_tab", st, k_pack_tab<<<(unsigned)tot, 256, 0, st>>>(m));
    return hipGetLastError();
}

hipError_t launch_set_refine_info_tab(bds_info* info, const int* ic, int K, hipStream_t st)
{
    if (K <= 0) return hipSuccess;
    BDS_TIMED("set_refine_info", st, k_set_refine_info_tab<<<(K + 255) / 256, 256, 0, st>>>(info, ic, K));
    return hipGetLastError();
}

hipError_t launch_clear_info(bds_info* info, int K, hipStream_t st)
{
    BDS_TIMED("clear_info", st, k_clear_info<<<(K + 255) / 256, 256, 0, st>>>(info, K));
    return hipGetLastError();
}

hipError_t launch_set_refine_info(bds_info* info, int iters, int converged, hipStream_t st)
{
    BDS_TIMED("set_refine_info", st, k_set_refine_info<<<1, 64, 0, st>>>(info, iters, converged));
    return hipGetLastError();
}

// explicit instantiations
#define BDS_INST_FAC(C, In)                                                                                   \
    template hipError_t launch_factor_level<C, In>(                                                           \
        const FacLv<Stor<C>::type, In>&, const FacLv<Stor<C>::type, In>*, const int64_t*, const int64_t*,    \
        const int64_t*, int, int64_t, int64_t, int64_t, int, const Tiling&, hipStream_t);
BDS_INST_FAC(double, double)
BDS_INST_FAC(float, double)
BDS_INST_FAC(float, float)
BDS_INST_FAC(bf16x, double)
BDS_INST_FAC(bf16x, float)
template hipError_t launch_coarse_factor<double>(const CoarseFac<double>&, const CoarseFac<double>*, int, int,
                                                 hipStream_t);
template hipError_t launch_coarse_factor<float>(const CoarseFac<float>&, const CoarseFac<float>*, int, int,
                                                hipStream_t);
template hipError_t launch_solve_fwd<double>(const SolLv<double>&, const SolLv<double>*, const int64_t*,
                                             const int64_t*, int, int64_t, int64_t, int, const Tiling&, hipStream_t);
template hipError_t launch_solve_fwd<float>(const SolLv<float>&, const SolLv<float>*, const int64_t*,
                                            const int64_t*, int, int64_t, int64_t, int, const Tiling&, hipStream_t);
template hipError_t launch_solve_bwd<double>(const SolLv<double>&, const SolLv<double>*, const int64_t*, int,
                                             int64_t, int, const Tiling&, hipStream_t);
template hipError_t launch_solve_bwd<float>(const SolLv<float>&, const SolLv<float>*, const int64_t*, int,
                                            int64_t, int, const Tiling&, hipStream_t);

}  // namespace bds
