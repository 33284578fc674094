// cellgeom.h -- fractional coordinates and cell index of a position in a
// slot's sheared box (internal; device code).
#pragma once

#include "engine.h"

namespace aqs {

// s = H^-1 r for the upper-triangular box H = [[Lx, t, 0], [0, Ly, 0], [0, 0, Lz]]
__device__ __forceinline__ void frac(const Geom& g, double t, double x, double y, double z,
                                     double* s) {
  s[1] = y / g.L[1];
  s[0] = (x - t * s[1]) / g.L[0];
  s[2] = z / g.L[2];
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int D>
__device__ __forceinline__ int cell_of_pos(const Geom& g, const int* nc, double t, const double4& p,
                                           int* c3) {
  double s[3];
  frac(g, t, p.x, p.y, (D == 3) ? p.z : 0.0, s);
  c3[0] = clampi((int)floor(s[0] * nc[0]), 0, nc[0] - 1);
  c3[1] = clampi((int)floor(s[1] * nc[1]), 0, nc[1] - 1);
  c3[2] = (D == 3) ? clampi((int)floor(s[2] * nc[2]), 0, nc[2] - 1) : 0;
  return (c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
}

}  // namespace aqs
