// cellgeom.h -- fractional coordinates and cell index of a position in a
// slot's deformed box (internal; device code).
#pragma once

#include "engine.h"

namespace aqs {

// s = H^-1 r: by back substitution for the upper-triangular box of simple
// shear, else by the adjugate of the (x, y) block (pure shear, Eq. 17)
__device__ __forceinline__ void frac(const Box& b, double x, double y, double z, double* s) {
  if (b.h10 == 0.0) {
    s[1] = y / b.h11;
    s[0] = (x - b.h01 * s[1]) / b.h00;
  } else {
    const double det = b.h00 * b.h11 - b.h01 * b.h10;
    s[0] = (b.h11 * x - b.h01 * y) / det;
    s[1] = (b.h00 * y - b.h10 * x) / det;
  }
  s[2] = z / b.h22;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int D>
__device__ __forceinline__ int cell_of_pos(const Box& b, const int* nc, const double4& p, int* c3) {
  double s[3];
  frac(b, p.x, p.y, (D == 3) ? p.z : 0.0, s);
  c3[0] = clampi((int)floor(s[0] * nc[0]), 0, nc[0] - 1);
  c3[1] = clampi((int)floor(s[1] * nc[1]), 0, nc[1] - 1);
  c3[2] = (D == 3) ? clampi((int)floor(s[2] * nc[2]), 0, nc[2] - 1) : 0;
  return (c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
}

}  // namespace aqs
