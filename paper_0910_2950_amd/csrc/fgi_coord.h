// Site coordinates on the checkerboarded lattice: parity, one periodic step
// along +-d, and the FP64 link U_d(y) at a coordinate.
#pragma once
#include "fgi_device.h"

namespace fgi {

__device__ __forceinline__ int coord_parity(const Coord& y) { return (y.c[0] + y.c[1] + y.c[2] + y.c[3]) & 1; }

__device__ __forceinline__ void coord_step(const Geom& g, Coord& y, int d, int fwd) {
    if (fwd) y.c[d] = y.c[d] + 1 == g.L[d] ? 0 : y.c[d] + 1;
    else y.c[d] = (y.c[d] == 0 ? g.L[d] : y.c[d]) - 1;
}

__device__ __forceinline__ M3<double> link_at(const Geom& g, const d2* U, int d, const Coord& y) {
    return gauge_load(U, d, coord_parity(y), cb_index(g, y), g.Vh);
}

}  // namespace fgi
