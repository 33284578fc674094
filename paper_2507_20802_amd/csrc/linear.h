// linear.h -- the linear-response start of an AQS step (Eqs. 7-8) on the
// device: conjugate gradients on H u = f(x0) at the plain start x0, with
// Hessian-vector products from central differences of the forces.
#pragma once

#include "engine.h"

namespace aqs {

// per 256-atom block: |r|^2, max |p_i|^2, p.Hp, max |u_i|^2, non-finite u
constexpr int kLinRR = 0, kLinPP = 1, kLinPHP = 2, kLinUU = 3, kLinBad = 4;

struct LinArgs {
  const int2* blocks;       // (slot, 256-atom block) table over the solving slots
  const int32_t* sel;       // the solving slots (per-slot kernels)
  int32_t nsel;
  int32_t it;               // solve iteration (parity of the residual norm buffer)
  const Geom* geom;
  State* state;
  LinState* lin;
  double4* pos4;            // the probes are written here (x0 restored at the end)
  const double4* x0;        // the plain start
  const double* fx; const double* fy; const double* fz;   // forces of the last evaluation
  double* ux; double* uy; double* uz;     // u (the start's displacement arrays)
  double* px; double* py; double* pz;     // search direction (velocities; zero after)
  double4* r4;              // residual r (free staging array)
  double* hx; double* hy; double* hz;     // f(x0 + s p), then H p (free staging arrays)
  double* part;             // per global block, kLearnParts doubles
  double probe;             // probe length h (max norm)
  double tol;               // stop when |r| <= tol |f(x0)|
  double max_move;          // largest accepted max_i |u_i|
};

// per slot: phase PH_LPROBE, solve scalars reset
void launch_lin_begin(const LinArgs& a, hipStream_t s);
// per block, forces f(x0) in place: r = p = f(x0), u = 0, partials |r|^2, max |p|^2
void launch_lin_init(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s);
// per slot: |r|^2 = |f(x0)|^2 into the solve scalars
void launch_lin_start(const LinArgs& a, hipStream_t s);
// per block: sign +1, x = x0 + s p; sign -1, keep f(x0 + s p), x = x0 - s p
// (s = h / max_i |p_i|)
void launch_lin_probe(const LinArgs& a, int32_t sign, int32_t nblk, int32_t dim, hipStream_t s);
// per block: H p from the two probes, partial p.Hp; then the update of u, r
// (partial |r|^2); then the new direction p (partial max |p_i|^2)
void launch_lin_hp(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s);
void launch_lin_update(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s);
void launch_lin_direction(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s);
// per block: x = x0, v = 0, partials max |u_i|^2 and non-finite u; then per
// slot: the pre-check, lmean = 0, phase PH_LPLAIN
void launch_lin_finish(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s);

}  // namespace aqs
