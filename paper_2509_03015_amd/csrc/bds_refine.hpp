// Stopping rule of the mixed-precision iterative refinement (host logic, no
// GPU dependency).
#pragma once

#include <cmath>

namespace bds {

// Stopping rule of the iterative refinement, given the norms of the latest
// correction (cn) and of the updated solution (xn), both Frobenius.  The
// corrections of classical refinement contract geometrically, by about
// rho = cn / prev per iteration, so after adding the latest correction the
// remaining error is about rho * cn.  Returns true when the iteration should
// stop and sets `converged`:
//   cn <= tol * xn, or (from the second iteration on) rho * cn <= tol * xn
//                                   -> converged
//   NaN                             -> diverged
//   cn > prev / 2 (not contracting) -> stop; converged iff cn <= 1e-8 * xn
// prev carries the previous correction norm (start with HUGE_VAL).
inline bool refine_stop(double cn, double xn, double& prev, double tol, int& converged)
{
    converged = 0;
    if (!(cn == cn) || !(xn == xn)) return true;
    const double rho = (prev < HUGE_VAL && prev > 0) ? cn / prev : 1.0;
    if (cn <= tol * xn || (rho < 0.5 && rho * cn <= tol * xn)) {
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
