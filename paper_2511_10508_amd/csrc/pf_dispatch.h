// Runtime -> compile-time dispatch helpers for the kernel families.
#pragma once

#include <type_traits>

#include "pf_internal.h"

namespace pf {

template <int... Rs> struct RList {};

// Calls f(std::integral_constant<int, R>) for the R of the list equal to r.
template <typename F, int R0, int... Rs>
bool dispatch_r(int r, RList<R0, Rs...>, F &&f)
{
    if (r == R0) {
        f(std::integral_constant<int, R0>{});
        return true;
    }
    if constexpr (sizeof...(Rs) > 0)
        return dispatch_r(r, RList<Rs...>{}, f);
    else
        return false;
}

template <typename F>
bool dispatch_kind(int kind, F &&f)
{
    switch (kind) {
    case kAC: f(std::integral_constant<int, kAC>{}); return true;
    case kCH: f(std::integral_constant<int, kCH>{}); return true;
    case kGS: f(std::integral_constant<int, kGS>{}); return true;
    case kMC: f(std::integral_constant<int, kMC>{}); return true;
    default: return false;
    }
}

// dispatch_kind plus the direct-biharmonic Cahn-Hilliard kernels (the
// families that have them: 1D, 2D fused, generic, reductions).
template <typename F>
bool dispatch_kind_all(int kind, F &&f)
{
    if (kind == kCHD) {
        f(std::integral_constant<int, kCHD>{});
        return true;
    }
    return dispatch_kind(kind, f);
}

// dispatch_kind_all plus Model H (the per-site generic kernels only).
template <typename F>
bool dispatch_kind_generic(int kind, F &&f)
{
    if (kind == kMH) {
        f(std::integral_constant<int, kMH>{});
        return true;
    }
    return dispatch_kind_all(kind, f);
}

template <typename F>
void dispatch_prec(int fp32, F &&f)
{
    if (fp32)
        f(float(0));
    else
        f(double(0));
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace pf
