// Host-side helpers shared by the single-system and batched entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "bds_plan.hpp"
#include "bds_refine.hpp"

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

}  // namespace bds
