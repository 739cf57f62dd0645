// Host-side helpers shared by the single-system and batched entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "bds_plan.hpp"

#define BDS_TRY(...)                           \
    do {                                       \
        hipError_t e_ = (__VA_ARGS__);         \
        if (e_ != hipSuccess) return BDS_EHIP; \
    } while (0)

namespace bds {

template <typename T> T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }
template <typename T> const T* at(const void* base, size_t off)
{
    return reinterpret_cast<const T*>(static_cast<const char*>(base) + off);
}

// Level-0 matrices in padded layout: the user's arrays, or their padded copies
// in the factor workspace when n is not a multiple of 16.
struct Level0 {
    const double* Ad;
    const double* As;
};

Level0 level0_matrices(const SysPlan& p, const double* Ad, const double* As, const void* fws);

// Stopping rule of the iterative refinement, given the norms of the latest
// correction (cn) and of the updated solution (xn), both Frobenius.  Returns
// true when the iteration should stop and sets `converged`:
//   cn <= tol * xn                  -> converged
//   NaN                             -> diverged
//   cn > prev / 2 (not contracting) -> stop; converged iff cn <= 1e-8 * xn
// prev carries the previous correction norm (start with HUGE_VAL).
inline bool refine_stop(double cn, double xn, double& prev, double tol, int& converged)
{
    converged = 0;
    if (!(cn == cn) || !(xn == xn)) return true;
    if (cn <= tol * xn) {
        converged = 1;
        return true;
    }
    if (cn > 0.5 * prev) {
        converged = cn <= 1e-8 * xn;
        return true;
    }
    prev = cn;
    return false;
}

}  // namespace bds
