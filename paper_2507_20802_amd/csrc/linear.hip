// linear.hip -- the linear-response start of an AQS step on gfx950.
//
// The equilibrium condition of Sec. 2.1 (Eqs. 7-8): an inherent structure
// strained by dgamma stays in equilibrium if its non-affine displacement
// solves H dr/dgamma = F~, F~ the force the affine deformation induces.
// After the affine step, the force at the plain start x0 = F r is F~ dgamma
// to first order, so the step's non-affine displacement is one Newton step
// from x0: H u = f(x0), H the Hessian of the energy at x0.  Conjugate
// gradients solve it with Hessian-vector products from central differences
// of the forces,
//   H p ~ (f(x0 - s p) - f(x0 + s p)) / (2 h) max_i |p_i|,  s = h / max_i |p_i|,
// each a pair of evaluations by the force kernel (slots in PH_LPROBE; the
// host drives the iterations).  The solve stops when |r|^2 <= tol^2 |f(x0)|^2,
// at non-positive curvature p.Hp <= 0 (no update), or after max_cg updates.
// The start x0 + u then goes through the learned start's checks: max_i |u_i|
// <= max_move, and E and max_i |F_i| no worse than at x0 (else x0).
//
// Each kernel takes one step of the iteration for every atom of the solving
// slots (one block per 256 atoms); sums over a slot's atoms are per-block
// partials combined over the blocks in a fixed order, the same in every
// block that needs them, so all blocks of a slot take the same decisions.
// The solve's scalars (LinState) are written by the owner block (block 0 of
// the slot) where no block of the same kernel reads them; the `done` flag
// is the exception, read as lin_item describes.
#include <hip/hip_runtime.h>

#include "learned.h"
#include "linear.h"

namespace aqs {

namespace {

// Entry c of the slot's per-block partials combined over its blocks (sum,
// or max if mx) in a fixed order; every thread of the block gets it.
__device__ double slot_total(const double* part, const Geom& g, int c, bool mx, double* red) {
  const int t = threadIdx.x;
  double v = 0.0;
  for (int b = t; b < g.nblocks; b += kBlock) {
    const double x = part[(int64_t)(g.block0 + b) * kLearnParts + c];
    v = mx ? fmax(v, x) : v + x;
  }
  red[t] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) red[t] = mx ? fmax(red[t], red[t + w]) : red[t] + red[t + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// The block's partial (sum, or max if mx) of v into entry c of its slot.
__device__ void block_part(double* part, int64_t blk, int c, double v, bool mx, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) red[t] = mx ? fmax(red[t], red[t + w]) : red[t] + red[t + w];
    __syncthreads();
  }
  if (t == 0) part[blk * kLearnParts + c] = red[0];
  __syncthreads();
}

// (slot, block) of this workgroup, or slot -1 if it has nothing to do: the
// slot must be solving (PH_LPROBE) and, unless `always`, not done.  One
// thread reads the flags and the block follows it: the owner block of the
// same kernel may set `done` meanwhile (on a decision every block takes
// alike), and the block must not split between its barriers.
__device__ int2 lin_item(const LinArgs& a, bool always) {
  __shared__ int go;
  const int2 bt = a.blocks[blockIdx.x];
  if (threadIdx.x == 0)
    go = (bt.x >= 0 && a.state[bt.x].phase == PH_LPROBE && (always || a.lin[bt.x].done == 0)) ? 1 : 0;
  __syncthreads();
  return go ? bt : make_int2(-1, 0);
}

__global__ __launch_bounds__(64) void k_lin_begin(LinArgs a) {
  if (threadIdx.x != 0) return;
  const int rep = a.sel[blockIdx.x];
  State* st = a.state + rep;
  if (st->phase != PH_LPLAIN) return;
  st->phase = PH_LPROBE;
  LinState& l = a.lin[rep];
  l.rr[0] = 0.0;
  l.rr[1] = 0.0;
  l.bb = 0.0;
  l.iters = 0;
  l.done = 0;
  l.probes = 0;
}

// forces f(x0) in place: r = p = f(x0), u = 0
template <int D>
__global__ __launch_bounds__(kBlock) void k_lin_init(LinArgs a) {
#pragma clang fp contract(off)
  const int2 bt = lin_item(a, true);
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  __shared__ double red[kBlock];
  const int li = bt.y * kBlock + threadIdx.x;
  double rr = 0.0;
  if (li < g.n) {
    const int64_t gi = g.atom_off + li;
    const double fx = a.fx[gi], fy = a.fy[gi], fz = (D == 3) ? a.fz[gi] : 0.0;
    a.r4[gi] = make_double4(fx, fy, fz, 0.0);
    a.px[gi] = fx;
    a.py[gi] = fy;
    if (D == 3) a.pz[gi] = fz;
    a.ux[gi] = 0.0;
    a.uy[gi] = 0.0;
    if (D == 3) a.uz[gi] = 0.0;
    rr = fx * fx + fy * fy + fz * fz;
  }
  const int64_t blk = g.block0 + bt.y;
  block_part(a.part, blk, kLinRR, rr, false, red);
  block_part(a.part, blk, kLinPP, rr, true, red);
}

__global__ __launch_bounds__(kBlock) void k_lin_start(LinArgs a) {
  const int rep = a.sel[blockIdx.x];
  if (a.state[rep].phase != PH_LPROBE) return;
  const Geom g = a.geom[rep];
  __shared__ double red[kBlock];
  const double rr = slot_total(a.part, g, kLinRR, false, red);
  if (threadIdx.x == 0) {
    a.lin[rep].rr[0] = rr;
    a.lin[rep].bb = rr;
  }
}

// sign +1: x = x0 + s p; sign -1: f(x0 + s p) kept, x = x0 - s p
template <int D>
__global__ __launch_bounds__(kBlock) void k_lin_probe(LinArgs a, int sign) {
#pragma clang fp contract(off)
  const int2 bt = lin_item(a, false);
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  __shared__ double red[kBlock];
  const double pmax = sqrt(slot_total(a.part, g, kLinPP, true, red));
  if (!(pmax > 0.0)) {   // p = 0: nothing to solve
    if (bt.y == 0 && threadIdx.x == 0) a.lin[bt.x].done = 1;
    return;
  }
  const double s = a.probe / pmax;
  const int li = bt.y * kBlock + threadIdx.x;
  if (li >= g.n) return;
  const int64_t gi = g.atom_off + li;
  if (sign < 0) {
    a.hx[gi] = a.fx[gi];
    a.hy[gi] = a.fy[gi];
    if (D == 3) a.hz[gi] = a.fz[gi];
  }
  const double4 x = a.x0[gi];
  const double px = a.px[gi], py = a.py[gi], pz = (D == 3) ? a.pz[gi] : 0.0;
  double4 q = x;
  if (sign > 0) {
    q.x = x.x + s * px;
    q.y = x.y + s * py;
    if (D == 3) q.z = x.z + s * pz;
  } else {
    q.x = x.x - s * px;
    q.y = x.y - s * py;
    if (D == 3) q.z = x.z - s * pz;
  }
  a.pos4[gi] = q;
}

// H p = (f(x0 - s p) - f(x0 + s p)) / (2 h) max_i |p_i| into h; partial p.Hp
template <int D>
__global__ __launch_bounds__(kBlock) void k_lin_hp(LinArgs a) {
#pragma clang fp contract(off)
  const int2 bt = lin_item(a, false);
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  __shared__ double red[kBlock];
  const double pmax = sqrt(slot_total(a.part, g, kLinPP, true, red));
  const double den = 2.0 * a.probe;
  const int li = bt.y * kBlock + threadIdx.x;
  double php = 0.0;
  if (li < g.n) {
    const int64_t gi = g.atom_off + li;
    const double hx = (a.fx[gi] - a.hx[gi]) / den * pmax;
    const double hy = (a.fy[gi] - a.hy[gi]) / den * pmax;
    const double hz = (D == 3) ? (a.fz[gi] - a.hz[gi]) / den * pmax : 0.0;
    a.hx[gi] = hx;
    a.hy[gi] = hy;
    if (D == 3) a.hz[gi] = hz;
    const double pz = (D == 3) ? a.pz[gi] : 0.0;
    php = a.px[gi] * hx + a.py[gi] * hy + pz * hz;
  }
  block_part(a.part, g.block0 + bt.y, kLinPHP, php, false, red);
  if (bt.y == 0 && threadIdx.x == 0) a.lin[bt.x].probes += 1;
}

// alpha = |r|^2 / p.Hp; u += alpha p; r -= alpha H p; partial |r|^2
template <int D>
__global__ __launch_bounds__(kBlock) void k_lin_update(LinArgs a) {
#pragma clang fp contract(off)
  const int2 bt = lin_item(a, false);
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  __shared__ double red[kBlock];
  const double php = slot_total(a.part, g, kLinPHP, false, red);
  if (!(php > 0.0)) {   // non-positive curvature: stop without an update
    if (bt.y == 0 && threadIdx.x == 0) a.lin[bt.x].done = 1;
    return;
  }
  const double alpha = a.lin[bt.x].rr[a.it & 1] / php;
  const int li = bt.y * kBlock + threadIdx.x;
  double rr = 0.0;
  if (li < g.n) {
    const int64_t gi = g.atom_off + li;
    a.ux[gi] = a.ux[gi] + alpha * a.px[gi];
    a.uy[gi] = a.uy[gi] + alpha * a.py[gi];
    if (D == 3) a.uz[gi] = a.uz[gi] + alpha * a.pz[gi];
    double4 r = a.r4[gi];
    r.x = r.x - alpha * a.hx[gi];
    r.y = r.y - alpha * a.hy[gi];
    if (D == 3) r.z = r.z - alpha * a.hz[gi];
    a.r4[gi] = r;
    rr = r.x * r.x + r.y * r.y + r.z * r.z;
  }
  block_part(a.part, g.block0 + bt.y, kLinRR, rr, false, red);
  if (bt.y == 0 && threadIdx.x == 0) a.lin[bt.x].iters += 1;
}

// converged if |r|^2 <= tol^2 |f(x0)|^2; else beta = |r|^2 / |r_old|^2,
// p = r + beta p; partial max |p_i|^2
template <int D>
__global__ __launch_bounds__(kBlock) void k_lin_direction(LinArgs a) {
#pragma clang fp contract(off)
  const int2 bt = lin_item(a, false);
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  LinState* l = a.lin + bt.x;
  __shared__ double red[kBlock];
  const double rrn = slot_total(a.part, g, kLinRR, false, red);
  if (rrn <= a.tol * a.tol * l->bb) {
    if (bt.y == 0 && threadIdx.x == 0) l->done = 1;
    return;
  }
  const double beta = rrn / l->rr[a.it & 1];
  const int li = bt.y * kBlock + threadIdx.x;
  double pp = 0.0;
  if (li < g.n) {
    const int64_t gi = g.atom_off + li;
    const double4 r = a.r4[gi];
    const double px = r.x + beta * a.px[gi];
    const double py = r.y + beta * a.py[gi];
    const double pz = (D == 3) ? r.z + beta * a.pz[gi] : 0.0;
    a.px[gi] = px;
    a.py[gi] = py;
    if (D == 3) a.pz[gi] = pz;
    pp = px * px + py * py + pz * pz;
  }
  block_part(a.part, g.block0 + bt.y, kLinPP, pp, true, red);
  if (bt.y == 0 && threadIdx.x == 0) l->rr[(a.it + 1) & 1] = rrn;
}

// x = x0, v = 0 (the direction's arrays); partials max |u_i|^2, non-finite u
template <int D>
__global__ __launch_bounds__(kBlock) void k_lin_finish(LinArgs a) {
#pragma clang fp contract(off)
  const int2 bt = lin_item(a, true);
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  __shared__ double red[kBlock];
  const int li = bt.y * kBlock + threadIdx.x;
  double uu = 0.0, bad = 0.0;
  if (li < g.n) {
    const int64_t gi = g.atom_off + li;
    a.pos4[gi] = a.x0[gi];
    a.px[gi] = 0.0;
    a.py[gi] = 0.0;
    if (D == 3) a.pz[gi] = 0.0;
    const double ux = a.ux[gi], uy = a.uy[gi], uz = (D == 3) ? a.uz[gi] : 0.0;
    const double q = ux * ux + uy * uy + uz * uz;
    if (isfinite(q)) {
      uu = q;
    } else {
      bad = 1.0;
    }
  }
  const int64_t blk = g.block0 + bt.y;
  block_part(a.part, blk, kLinUU, uu, true, red);
  block_part(a.part, blk, kLinBad, bad, true, red);
}

// the pre-check of the start (finite, max_i |u_i| <= max_move), lmean = 0
// (the move adds u itself), phase PH_LPLAIN
__global__ __launch_bounds__(kBlock) void k_lin_ctl(LinArgs a) {
  const int rep = a.sel[blockIdx.x];
  State* st = a.state + rep;
  if (st->phase != PH_LPROBE) return;
  const Geom g = a.geom[rep];
  __shared__ double red[kBlock];
  const double uu = slot_total(a.part, g, kLinUU, true, red);
  const double bad = slot_total(a.part, g, kLinBad, true, red);
  if (threadIdx.x == 0) {
    st->learn_ok = (bad == 0.0 && sqrt(uu) <= a.max_move) ? 1 : 0;
    st->lmean[0] = 0.0;
    st->lmean[1] = 0.0;
    st->lmean[2] = 0.0;
    st->phase = PH_LPLAIN;
  }
}

}  // namespace

void launch_lin_begin(const LinArgs& a, hipStream_t s) {
  if (a.nsel > 0) hipLaunchKernelGGL(k_lin_begin, dim3(a.nsel), dim3(64), 0, s, a);
}

void launch_lin_init(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s) {
  if (nblk <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_lin_init<3>, dim3(nblk), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_lin_init<2>, dim3(nblk), dim3(kBlock), 0, s, a);
}

void launch_lin_start(const LinArgs& a, hipStream_t s) {
  if (a.nsel > 0) hipLaunchKernelGGL(k_lin_start, dim3(a.nsel), dim3(kBlock), 0, s, a);
}

void launch_lin_probe(const LinArgs& a, int32_t sign, int32_t nblk, int32_t dim, hipStream_t s) {
  if (nblk <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_lin_probe<3>, dim3(nblk), dim3(kBlock), 0, s, a, (int)sign);
  else
    hipLaunchKernelGGL(k_lin_probe<2>, dim3(nblk), dim3(kBlock), 0, s, a, (int)sign);
}

void launch_lin_hp(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s) {
  if (nblk <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_lin_hp<3>, dim3(nblk), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_lin_hp<2>, dim3(nblk), dim3(kBlock), 0, s, a);
}

void launch_lin_update(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s) {
  if (nblk <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_lin_update<3>, dim3(nblk), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_lin_update<2>, dim3(nblk), dim3(kBlock), 0, s, a);
}

void launch_lin_direction(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s) {
  if (nblk <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_lin_direction<3>, dim3(nblk), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_lin_direction<2>, dim3(nblk), dim3(kBlock), 0, s, a);
}

void launch_lin_finish(const LinArgs& a, int32_t nblk, int32_t dim, hipStream_t s) {
  if (nblk > 0) {
    if (dim == 3)
      hipLaunchKernelGGL(k_lin_finish<3>, dim3(nblk), dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL(k_lin_finish<2>, dim3(nblk), dim3(kBlock), 0, s, a);
  }
  if (a.nsel > 0) hipLaunchKernelGGL(k_lin_ctl, dim3(a.nsel), dim3(kBlock), 0, s, a);
}

}  // namespace aqs
