// Sliced ELLPACK (SELL-C-sigma) slice kernel launcher (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"
#include "launch.h"

namespace spmvlib {

// Launches the slice kernel of a SELL handle (long rows are launched by the
// caller): y[perm[slot]] = sum over the slot's entries, epilogue `epi`
// (EPI_PLAIN, EPI_DOT or EPI_RESID) with one partial per workgroup in
// g.part[0 .. M.n_sell_wg).
template <typename V, typename X, typename Y, typename A>
void launch_sell_slices(const DevMatrix &M, SpmvArgs<V, X, Y> g, int epi, hipStream_t st);

}  // namespace spmvlib
