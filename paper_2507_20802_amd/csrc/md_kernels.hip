// md_kernels.hip -- gfx950 kernels of the AQS hot path: cell binning and
// neighbour lists, the FP64 Lennard-Jones force loop with the per-slot FIRE
// control, the FIRE update, affine shear, configuration comparison, stress.
//
// Method: Reihn, Bamer, Stamm, arXiv 2507.20802.  Pair potential Eq. (13);
// affine simple shear Eqs. (2), (3), (16); minimisation operator Eq. (10)
// realised by FIRE 2.0; equality test Eq. (20); AQS chain Eqs. (12), (19).
//
// Determinism: no floating-point atomics.  Per-block partial sums use a fixed
// butterfly per wavefront and a fixed order across wavefronts; the last
// block of a slot combines the partials in block order.  Cell order within a
// cell is by atom id, so a rebuild gives the same sorted order every run.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>

#include "cellgeom.h"
#include "kernels.h"
#include "tiles.h"

namespace aqs {

// ---------------------------------------------------------------------------
// reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Block-wide reduction of NV values over NW wavefronts; op[c] = 0 sum,
// 1 max.  Result valid in thread 0.  Fixed order: butterfly inside each
// wavefront, then a pairwise tree over the wavefronts in index order.
template <int NV, int NW = kBlock / kWave>
__device__ __forceinline__ void block_reduce(double* v, const int* op, double (*lds)[NW]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = op[c] ? wave_max(v[c]) : wave_sum(v[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) lds[c][w] = v[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double t[NW];
#pragma unroll
      for (int i = 0; i < NW; ++i) t[i] = lds[c][i];
#pragma unroll
      for (int h = 1; h < NW; h <<= 1)
#pragma unroll
        for (int i = 0; i + h < NW; i += 2 * h) t[i] = op[c] ? fmax(t[i], t[i + h]) : t[i] + t[i + h];
      v[c] = t[0];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// box geometry: H = box_at(g, k) (engine.h): simple shear [[Lx, t, 0], [0, Ly,
// 0], [0, 0, Lz]], t = gamma Ly (Eq. 1, Eq. 16), or the pure shear of Eq. (17).
// Image code c = (ix+1) + 3 (iy+1) + 9 (iz+1); shift = H (ix, iy, iz).



// ---------------------------------------------------------------------------
// Lennard-Jones pair loop of one atom over its neighbour list, Eq. (13).
// Accumulates F_i = sum_j U'(r) d / r (d = r_j - r_i) and, if WE, the pair
// energy sum_j U(r) and sum_j U'(r) dx dy / r; the caller halves pair sums.
//
// The list is walked in chunks of kChunk entries: the chunk's neighbour
// positions are gathered together while the next chunk's list entries are
// already in flight, so one wavefront keeps 2 kChunk loads outstanding
// instead of waiting on two dependent loads per pair.  1/r^2 is the hardware
// reciprocal estimate refined by two Newton-Raphson steps (r <- r (2 - x r)),
// within 1 ulp of the rounded quotient.

constexpr int kChunk = 2;
// Fourth word of a buffer resource on gfx9-family GPUs (raw 32-bit data,
// offsets in bytes).
constexpr int kBufferFlags = 0x00020000;
// Coordinate of the far fill slot, the last LDS halo slot: list entries past
// a lane's count name it, and its distance from any atom is beyond every cutoff.
constexpr double kFarFill = 1.0e20;

__device__ __forceinline__ double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// One pair term, branch-free: out-of-range pairs contribute exact zeros (the
// result is selected away), so the kChunk pairs of a chunk interleave
// without divergence.  SAFE: the entry may be this atom itself or a stale
// fill entry (distance 0), so it is masked by `live` and its 1/r^2 taken of
// 1.0; otherwise every entry is another atom or the far fill slot, at a
// positive distance.  U'(r)/r = eps4 s6 (6 - 12 s6) / r^2 with s6 = (s/r)^6.
template <int D, bool WE, bool SAFE>
__device__ __forceinline__ void pair_term(bool live, double dx, double dy, double dz,
                                          const PairParams& q, double& fx, double& fy, double& fz,
                                          double& e, double& w) {
  const double r2 = (D == 3) ? dx * dx + dy * dy + dz * dz : dx * dx + dy * dy;
  const bool in = SAFE ? (live && (r2 < q.rc2)) : (r2 < q.rc2);
  const double inv = recip_nr(SAFE ? (in ? r2 : 1.0) : r2);
  const double s2 = q.sig2 * inv;
  const double s6 = s2 * s2 * s2;
  const double gv = s6 * fma(-12.0 * q.eps4, s6, 6.0 * q.eps4) * inv;
  const double g = in ? gv : 0.0;
  fx += g * dx;
  fy += g * dy;
  if (D == 3) fz += g * dz;
  if (WE) {
    e += in ? q.eps4 * (s6 * s6 - s6) - q.ucut : 0.0;
    w += g * dx * dy;
  }
}

// Halo coordinate at byte offset `off` (an LDS list entry).
__device__ __forceinline__ double lds_at(const double* h, uint32_t off) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(h) + off);
}

// Entry k of this lane's share of a list (rows sub, sub + TPA, ...), read
// as a buffer load from the slot's list: the step kk is clamped below the
// list capacity kcap, so the byte offset splits into a wave-uniform part
// sb + kk ss (scalar offset) and the lane's fixed part lb (vector offset)
// and needs no per-lane address arithmetic; entries past the lane's count
// become `fill`.  Offsets are taken modulo 2^32 (ss < 0 for B segments).
__device__ __forceinline__ uint32_t list_entry(__amdgpu_buffer_rsrc_t rs, uint32_t lb, uint32_t sb,
                                               uint32_t ss, int k, int my, int kcap,
                                               uint32_t fill) {
  const uint32_t kk = (uint32_t)min(k, kcap - 1);
  const uint32_t raw = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)lb, (int)(sb + kk * ss), 0);
  return k < my ? raw : fill;
}

// One segment of a word list (a tile without an LDS halo): this lane's
// entry k (k = 0 .. my - 1) sits at byte offset lb + sb + k ss of the slot's
// list (ss < 0 walks the B segment down from the top) and holds
// j | image code << 24; all neighbours of the segment have the same type, so
// the pair parameters q are fixed.
template <int D, bool WE, int TPA>
__device__ __forceinline__ void pair_segment(const double4 pi, __amdgpu_buffer_rsrc_t rs,
                                             uint32_t lb, uint32_t sb, uint32_t ss, int my,
                                             int kcap, uint32_t fill,
                                             const PairParams q, const double4* __restrict__ P,
                                             const double (*sh)[4], double& fx, double& fy,
                                             double& fz, double& e, double& w) {
  uint32_t cur[kChunk];
#pragma unroll
  for (int u = 0; u < kChunk; ++u) cur[u] = list_entry(rs, lb, sb, ss, u, my, kcap, fill);
  for (int k0 = 0; k0 < my; k0 += kChunk) {
    double4 pj[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) pj[u] = P[cur[u] & kIdxMask];
    uint32_t nxt[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      nxt[u] = list_entry(rs, lb, sb, ss, k0 + kChunk + u, my, kcap, fill);
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const uint32_t ent = cur[u];
      const int code = (int)((ent >> kCodeShift) & 31u);
      const double dx = (pj[u].x - pi.x) + sh[code][0];
      const double dy = (pj[u].y - pi.y) + sh[code][1];
      const double dz = (D == 3) ? (pj[u].z - pi.z) + sh[code][2] : 0.0;
      pair_term<D, WE, true>(k0 + u < my, dx, dy, dz, q, fx, fy, fz, e, w);
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) cur[u] = nxt[u];
  }
}

// Combine the TPA lanes of an atom (fixed butterfly: every lane of the group
// ends with the same bits).
template <int D, bool WE, int TPA>
__device__ __forceinline__ void combine_lanes(double& fx, double& fy, double& fz, double& e,
                                              double& w) {
#pragma unroll
  for (int off = 1; off < TPA; off <<= 1) {
    fx += __shfl_xor(fx, off, kWave);
    fy += __shfl_xor(fy, off, kWave);
    if (D == 3) fz += __shfl_xor(fz, off, kWave);
    if (WE) {
      e += __shfl_xor(e, off, kWave);
      w += __shfl_xor(w, off, kWave);
    }
  }
}

// Lennard-Jones sum of one atom over its word list, TPA lanes per atom.  The
// list (engine.h) holds the nA neighbours of type A in rows 0 .. nA - 1 and
// the nB of type B in rows max_nb - 1 down to max_nb - nB; lane sub takes
// rows sub, sub + TPA, ... of each.
template <int D, bool WE, int TPA>
__device__ __forceinline__ void atom_pairs(const double4 pi, int ti, const uint32_t* __restrict__ Ls,
                                           int col, int64_t stride, int32_t counts, int max_nb,
                                           uint32_t fill, const double4* __restrict__ P,
                                           const double (*sh)[4], const PairParams* pp, double& fx,
                                           double& fy, double& fz, double& e, double& w) {
  const int sub = (int)(threadIdx.x % TPA);
  const int na = counts & 0xffff, nb = (counts >> 16) & 0xffff;
  const int kcap = max_nb / TPA;
  const int my_a = na > sub ? (na - sub + TPA - 1) / TPA : 0;
  const int my_b = nb > sub ? (nb - sub + TPA - 1) / TPA : 0;
  // Row of step k: A  k TPA + sub,  B  max_nb - 1 - sub - k TPA
  //   = (max_nb - TPA - k TPA) + (TPA - 1 - sub); the first term is
  // wave-uniform (scalar offset), the second the lane's (vector offset).
  // Byte offsets stay below 2^32: a slot's list has under 2^30 words.
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint32_t*>(Ls), (short)0, (int)(4u * (uint32_t)stride * (uint32_t)max_nb),
      kBufferFlags);
  const uint32_t row_bytes = 4u * (uint32_t)stride;
  const uint32_t step = (uint32_t)TPA * row_bytes;
  const uint32_t lba = 4u * (uint32_t)col + (uint32_t)sub * row_bytes;
  const uint32_t lbb = 4u * (uint32_t)col + (uint32_t)(TPA - 1 - sub) * row_bytes;
  pair_segment<D, WE, TPA>(pi, rs, lba, 0u, step, my_a, kcap, fill, pp[2 * ti], P, sh, fx, fy, fz,
                           e, w);
  pair_segment<D, WE, TPA>(pi, rs, lbb, (uint32_t)(max_nb - TPA) * row_bytes, 0u - step, my_b,
                           kcap, fill, pp[2 * ti + 1], P, sh, fx, fy, fz, e, w);
  combine_lanes<D, WE, TPA>(fx, fy, fz, e, w);
}

// Cache policy of the packed-list loads: the default (cached in L2).  The
// lists stay the same between rebuilds, hundreds of iterations, and with
// each lane loading only its own groups a 16-replica batch keeps enough of
// them in the XCDs' L2s: 67 against 73 us per launch with non-temporal
// loads; one replica runs within 1 % either way.
constexpr int kListCachePolicy = 0;

// Group k of this lane's share of a packed list segment: the 8 bytes (four
// 16-bit entries) at byte offset lb + sb + k ss, k clamped below gcap so the
// scalar part sb + k ss stays wave-uniform and inside the slot's list.
__device__ __forceinline__ uint2 packed_group(__amdgpu_buffer_rsrc_t rs, uint32_t lb, uint32_t sb,
                                              uint32_t ss, int k, int gcap) {
  const uint32_t kk = (uint32_t)min(k, gcap - 1);
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)lb, (int)(sb + kk * ss),
                                                      kListCachePolicy);
  return make_uint2(v[0], v[1]);
}

// One pair from the LDS halo: `off` is the byte offset of the neighbour's
// halo slot (another atom, or the far fill slot: always a positive
// distance).
template <int D, bool WE>
__device__ __forceinline__ void halo_pair(uint32_t off, const double4& pi, const double* hx,
                                          const double* hy, const double* hz, const PairParams& q,
                                          double& fx, double& fy, double& fz, double& e,
                                          double& w) {
  const double dx = lds_at(hx, off) - pi.x;
  const double dy = lds_at(hy, off) - pi.y;
  const double dz = (D == 3) ? lds_at(hz, off) - pi.z : 0.0;
  pair_term<D, WE, false>(true, dx, dy, dz, q, fx, fy, fz, e, w);
}

// One segment of a packed list: this lane's groups k = 0 .. my - 1, each
// summed while the next one is in flight (one group ahead: measured on one
// 32768-atom replica and on a batch of 16, 3D, two lanes per atom, deeper
// prefetch is no faster).  `next` is the segment's first group, requested
// by the caller together with the other segment's, so that neither segment
// starts on a cold load; only the lane's own groups are loaded.
template <int D, bool WE>
__device__ __forceinline__ void packed_segment(const double4 pi, __amdgpu_buffer_rsrc_t rs,
                                               uint32_t lb, uint32_t sb, uint32_t ss, int my,
                                               int gcap, uint2 next, const PairParams q,
                                               const double* hx, const double* hy,
                                               const double* hz, double& fx, double& fy,
                                               double& fz, double& e, double& w) {
  for (int k = 0; k < my; ++k) {
    const uint2 cur = next;
    if (k + 1 < my) next = packed_group(rs, lb, sb, ss, k + 1, gcap);
    halo_pair<D, WE>(cur.x & 0xffffu, pi, hx, hy, hz, q, fx, fy, fz, e, w);
    halo_pair<D, WE>(cur.x >> 16, pi, hx, hy, hz, q, fx, fy, fz, e, w);
    halo_pair<D, WE>(cur.y & 0xffffu, pi, hx, hy, hz, q, fx, fy, fz, e, w);
    halo_pair<D, WE>(cur.y >> 16, pi, hx, hy, hz, q, fx, fy, fz, e, w);
  }
}

// Lennard-Jones sum of one atom over its packed list (engine.h), TPA lanes
// per atom: lane sub takes the A groups sub, sub + TPA, ... from group row 0
// up and the B groups from group row G - 1 - sub down (G = max_nb / 4).
template <int D, bool WE, int TPA>
__device__ __forceinline__ void atom_pairs_packed(const double4 pi, int ti, const uint2* Lp, int col,
                                                  int npad, int32_t counts, int max_nb,
                                                  const double* hx, const double* hy,
                                                  const double* hz, const PairParams* pp,
                                                  double& fx, double& fy, double& fz, double& e,
                                                  double& w) {
  const int sub = (int)(threadIdx.x % TPA);
  const int G = max_nb / kGroup;
  const int na = counts & 0xffff, nb = (counts >> 16) & 0xffff;
  const int ga = (na + kGroup - 1) / kGroup, gb = (nb + kGroup - 1) / kGroup;
  const int gcap = G / TPA;
  const int my_a = ga > sub ? (ga - sub + TPA - 1) / TPA : 0;
  const int my_b = gb > sub ? (gb - sub + TPA - 1) / TPA : 0;
  // group row of step k: A  k TPA + sub,  B  (G - TPA - k TPA) + (TPA - 1 - sub)
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint2*>(Lp), (short)0, (int)(8u * (uint32_t)npad * (uint32_t)G), kBufferFlags);
  const uint32_t row_bytes = 8u * (uint32_t)npad;
  const uint32_t step = (uint32_t)TPA * row_bytes;
  const uint32_t lba = 8u * (uint32_t)col + (uint32_t)sub * row_bytes;
  const uint32_t lbb = 8u * (uint32_t)col + (uint32_t)(TPA - 1 - sub) * row_bytes;
  const uint32_t sbb = (uint32_t)(G - TPA) * row_bytes;
  const uint2 first_a = my_a > 0 ? packed_group(rs, lba, 0u, step, 0, gcap) : make_uint2(0u, 0u);
  const uint2 first_b = my_b > 0 ? packed_group(rs, lbb, sbb, 0u - step, 0, gcap) : make_uint2(0u, 0u);
  packed_segment<D, WE>(pi, rs, lba, 0u, step, my_a, gcap, first_a, pp[2 * ti], hx, hy, hz, fx, fy,
                        fz, e, w);
  packed_segment<D, WE>(pi, rs, lbb, sbb, 0u - step, my_b, gcap, first_b, pp[2 * ti + 1], hx, hy, hz,
                        fx, fy, fz, e, w);
  combine_lanes<D, WE, TPA>(fx, fy, fz, e, w);
}

// ---------------------------------------------------------------------------
// Per-slot FIRE control, run by thread 0 of the last block of a slot after
// the force evaluation (Eq. 10 realised by FIRE 2.0; chain of Eq. 19).
//
// The force loop skips the pair energy during FIRE iterations (FIRE needs
// only forces).  A minimisation that ends, or reaches max_iter, goes through
// PH_ENERGY: one more evaluation at the same positions that also sums the
// energy and the shear virial, after which the pending outcome is recorded.

// Field-by-field copy of a slot state: an aggregate copy of the struct goes
// through scratch memory, a round trip on the control's critical path.
static_assert(sizeof(State) == 232, "copy_state copies every field of State");
__device__ __forceinline__ void copy_state(State& d, const State& s) {
  d.k = s.k;
  d.it = s.it;
  d.dt = s.dt;
  d.alpha = s.alpha;
  d.cv = s.cv;
  d.cf = s.cf;
  d.E = s.E;
  d.fmax = s.fmax;
  d.sxy = s.sxy;
  d.ubound = s.ubound;
  d.gamma_build = s.gamma_build;
  d.E_plain = s.E_plain;
  d.fmax_plain = s.fmax_plain;
  d.lmean[0] = s.lmean[0];
  d.lmean[1] = s.lmean[1];
  d.lmean[2] = s.lmean[2];
  d.npos = s.npos;
  d.nneg = s.nneg;
  d.restart = s.restart;
  d.phase = s.phase;
  d.status = s.status;
  d.step = s.step;
  d.n_steps = s.n_steps;
  d.snap_dst = s.snap_dst;
  d.do_snap = s.do_snap;
  d.nc[0] = s.nc[0];
  d.nc[1] = s.nc[1];
  d.nc[2] = s.nc[2];
  d.start_mode = s.start_mode;
  d.start_used = s.start_used;
  d.learn_ok = s.learn_ok;
  d.pending = s.pending;
  d.tiles_x = s.tiles_x;
  d.ntiles = s.ntiles;
  d.list_mode = s.list_mode;
  d.resume_phase = s.resume_phase;
  d.drops = s.drops;
  d.sxy_prev = s.sxy_prev;
  d.k_build = s.k_build;
}

// End of a minimisation with the given status: the step record, the
// snapshot slot's scalars, then the next fine step of the chain or the
// finish.  owner: this block records (every block of the slot computes the
// same new state; one of them writes what lives outside it).
__device__ __forceinline__ void finish_min(const IterArgs& a, int rep, State& s, int status,
                                           bool owner) {
  if (owner && s.step < a.log_cap) {
    StepRecord* rec = a.log + (int64_t)rep * a.log_cap + s.step;
    rec->iters = s.it;
    rec->energy = s.E;
    rec->max_f = s.fmax;
    rec->sigma_xy = s.sxy;
    rec->status = status;
    rec->start = s.start_used;
  }
  // a fine step whose inherent structure carries less shear stress than the
  // one before: under growing shear an elastic branch only gains stress, so
  // this marks a plastic event (aqs_run_round with live = 2 reads it)
  if (status == 0) {
    if (s.step >= 1 && s.sxy < s.sxy_prev) s.drops += 1;
    s.sxy_prev = s.sxy;
  }
  s.status = status;
  s.do_snap = (s.step == 0 && s.snap_dst >= 0) ? 1 : 0;
  if (s.do_snap && owner) {
    // the snapshot slot is not in the launch, so its state lives in the home buffer
    State* d = a.state_home + s.snap_dst;
    d->k = s.k;
    d->E = s.E;
    d->fmax = s.fmax;
    d->sxy = s.sxy;
    d->status = status;
  }
  if (status == 0 && s.step < s.n_steps) {
    s.step += 1;
    s.dt = a.fire.dt0;
    s.alpha = a.fire.alpha0;
    s.npos = 0;
    s.nneg = 0;
    s.it = 0;
    s.restart = 0;
    s.cv = 1.0;
    s.cf = 0.0;
    if (predicted_start_mode(s.start_mode)) {
      // the predicted displacement at this inherent structure first (the
      // network, the extrapolation or the linear response); the strain
      // index advances with the plain start (learned kernels)
      s.start_used = kStartFallback;
      s.phase = PH_LDESC;
    } else {
      s.k += 1;
      s.start_used = kStartPlain;
      s.phase = PH_ADVANCE;
    }
  } else {
    s.phase = PH_FINISH;
  }
}

// Conjugate-gradient control (Eq. 10 by the paper's own minimiser, Sec. 2.1):
// Polak-Ribiere with beta >= 0, and a line search on the directional
// derivative phi'(a) = -F(x0 + a d).d alone (no energies) that stops at the
// nearest minimum along d.  One evaluation per iteration; the update kernel
// then either starts a new direction (d = F + beta d, F0 = F, x += a1 d) or
// moves to the next trial (x += (a' - a) d).  Steps 3-6 of the minimiser:
//   3  p = phi'(a); the search ends if |p| <= sigma |p0| or, still
//      descending, the step has reached a_max = dmax / max_i |d_i|; then
//      beta = max(0, (|F|^2 - F.F0) / |F0|^2)
//   4  after ls_max evaluations in one search: beta = 0 (steepest descent);
//      more than n_fail_max such failures in a row: STALLED
//   5  next trial: secant extrapolation from the last two descending points,
//      kept in [1.1 a, grow a] and under a_max; once a point past the
//      minimum exists, the secant root of the bracket, kept in its middle 80 %
//   6  new direction: F.d = |F|^2 - beta p (beta = 0 unless positive);
//      first trial a_prev p0_prev / p0 (a_init for the first search and after
//      a failed one), at most dmax / (max|F_i| + beta max|d_i|)
// r: [1] |F|^2, [2] F.d, [3] F.F0, [8] max |d_i|^2; fmx = max_i |F_i|; it =
// iterations of this minimisation so far (0: reset the search state).
// Returns false if the minimisation has stalled.
__device__ bool control_cg(const CgParams& c, CgState& q, double fmx, int64_t it,
                           const double* r) {
#pragma clang fp contract(off)
  if (it == 0) {  // first evaluation of a minimisation
    q.dir = 0;
    q.nfail = 0;
    q.aprev = 0.0;
  }
  const double ff = r[1];
  double beta = 0.0, p = 0.0, dn = 0.0;
  if (q.dir) {
    p = -r[2];
    dn = sqrt(r[8]);
    const double a_max = c.dmax / dn;
    if (fabs(p) <= c.sigma * fabs(q.p0) || (p < 0.0 && q.a >= a_max)) {
      beta = fmax(0.0, (ff - r[3]) / q.ff0);
      q.aprev = q.a;
      q.p0prev = q.p0;
      q.nfail = 0;
    } else if (++q.nls > c.ls_max) {
      if (++q.nfail > c.n_fail_max) return false;
      q.aprev = 0.0;
    } else {
      const double at = q.a, a_old = q.alo, p_old = q.plo;
      if (p < 0.0) {
        q.alo = at;
        q.plo = p;
      } else {
        q.ahi = at;
        q.phi = p;
      }
      double an;
      if (q.ahi < 0.0) {
        an = c.grow * at;
        if (p > p_old) an = fmin(fmax(at - p * (at - a_old) / (p - p_old), 1.1 * at), c.grow * at);
        an = fmin(an, a_max);
      } else {
        const double w = q.ahi - q.alo;
        an = fmin(fmax(q.alo - q.plo * w / (q.phi - q.plo), q.alo + 0.1 * w),
                  q.ahi - 0.1 * w);
      }
      q.newdir = 0;
      q.step = an - at;
      q.a = an;
      return true;
    }
  }
  double fd = ff - beta * p;
  if (!(fd > 0.0)) beta = 0.0;
  if (beta == 0.0) fd = ff;
  double a1 = (q.aprev > 0.0) ? q.aprev * q.p0prev / (-fd) : c.a_init;
  const double cap = c.dmax / (fmx + beta * dn);
  if (a1 > cap) a1 = cap;
  q.newdir = 1;
  q.beta = beta;
  q.step = a1;
  q.p0 = -fd;
  q.ff0 = ff;
  q.a = a1;
  q.alo = 0.0;
  q.plo = -fd;
  q.ahi = -1.0;
  q.nls = 0;
  q.dir = 1;
  return true;
}

// The control of one iteration from the slot's sums r: advances the slot's
// state s and conjugate-gradient state q in place (owner: this block writes
// the records, see finish_min).
template <bool CG>
__device__ __forceinline__ void control(const IterArgs& a, int rep, const Geom& g, const double* r,
                                        int phase, State& s, CgState& q, bool owner) {
  // written-out arithmetic only (no fused multiply-adds): the control's
  // rounding does not depend on where the compiler keeps the state
#pragma clang fp contract(off)
  if (phase == PH_FINISH || phase == PH_STOP) {
    s.phase = PH_DONE;
    return;
  }
  // Validity of the neighbour list.  With r_i = F x_ref,i + u_i (F the shear
  // since the build, |gamma - gamma_build| = gd) every pair now closer than
  // its cutoff was within cutoff + skin at the build if
  //   gd rc_max + 2 (1 + gd) max_i |u_i| < skin
  // (simple shear; the pure shear bounds it by the norm of F^-1).
  const double ub = r[7];
  constexpr bool cg = CG;
  bool valid;
  if (g.dgamma_y == 0.0) {
    const double gam = strain_of(s.k, g.dgamma);
    const double gd = fabs(gam - s.gamma_build);
    valid = gd * a.rc_max + 2.0 * (1.0 + gd) * ub < a.skin;
  } else {
    // pure shear: r_i = G x_ref,i + u_i with G = H_k H_build^-1, so a pair now
    // closer than its cutoff had |d_build| <= |G^-1| (rc + 2 max |u_i|)
    valid = inverse_strain_norm(g, s.k, s.k_build) * (a.rc_max + 2.0 * ub) < a.rc_max + a.skin;
  }
  if (!valid) {
    s.resume_phase = (phase == PH_LPLAIN || phase == PH_LMOVE || phase == PH_LREVERT)
                         ? phase
                         : (cg ? PH_CG : PH_FIRE);
    s.phase = PH_REBUILD;
    return;
  }
  s.ubound = ub;
  s.fmax = sqrt(r[4]);
  if (phase == PH_EVAL || phase == PH_ENERGY) {
    s.E = r[0];
    if (g.dgamma_y == 0.0) {
      s.sxy = r[5] / (g.L[0] * g.L[1] * g.L[2]);  // simple shear keeps V = Lx Ly Lz
    } else {
      const Box bx = box_at(g, s.k);   // the pure shear scales the (x, y) area
      s.sxy = r[5] / (fabs(bx.h00 * bx.h11 - bx.h01 * bx.h10) * bx.h22);
    }
    if (phase == PH_EVAL) {
      s.phase = PH_DONE;
    } else if (s.pending == 1) {  // max_iter reached: record, then apply the last step
      finish_min(a, rep, s, 1, owner);
      s.phase = PH_STOP;
    } else {
      finish_min(a, rep, s, s.pending, owner);
    }
    return;
  }
  // learned start: the plain start's E and max |F| are the reference; the
  // learned start is kept only if it is no worse in both, else reverted
  if (phase == PH_LPLAIN) {
    s.E_plain = r[0];
    s.fmax_plain = s.fmax;
    if (s.learn_ok && r[6] == 0.0 && isfinite(r[0]) && isfinite(r[4])) {
      s.phase = PH_LMOVE;
      return;
    }
    s.start_used = kStartFallback;
  } else if (phase == PH_LMOVE) {
    const bool worse = r[6] != 0.0 || !isfinite(r[0]) || !isfinite(r[4]) ||
                       r[0] > s.E_plain || s.fmax > s.fmax_plain;
    if (worse) {
      s.start_used = kStartFallback;
      s.phase = PH_LREVERT;
      return;
    }
    s.start_used = s.start_mode;   // the predicted start is kept
  }
  s.phase = cg ? PH_CG : PH_FIRE;
  if (r[6] != 0.0 || !isfinite(r[1]) || !isfinite(r[2])) {
    s.E = NAN;
    s.sxy = NAN;
    finish_min(a, rep, s, 3, owner);
    return;
  }
  if (s.fmax < (cg ? a.cg.ftol : a.fire.ftol)) {
    s.pending = 0;
    s.phase = PH_ENERGY;
    return;
  }
  if (cg) {
    const bool going = control_cg(a.cg, q, s.fmax, s.it, r);
    if (!going) {
      s.pending = 2;
      s.phase = PH_ENERGY;
    } else {
      s.it += 1;
      if (s.it >= a.cg.max_iter) {
        s.pending = 1;
        s.phase = PH_ENERGY;  // energy at these positions, then the last step
      }
    }
    return;
  }
  const FireParams& f = a.fire;
  const double FF = r[1], P = r[2], VV = r[3];
  if (P > 0.0) {
    s.npos += 1;
    s.nneg = 0;
    if (s.npos > f.n_delay) {
      s.dt = fmin(s.dt * f.f_inc, f.dt_max);
      s.alpha *= f.f_alpha;
    }
    s.restart = 0;
  } else {
    s.npos = 0;
    s.nneg += 1;
    if (s.nneg > f.n_neg_max) {
      s.pending = 2;
      s.phase = PH_ENERGY;
      return;
    }
    if (!(f.initial_delay && s.it < f.n_delay)) {
      if (s.dt * f.f_dec >= f.dt_min) s.dt *= f.f_dec;
      s.alpha = f.alpha0;
    }
    s.restart = 1;
  }
  // |v|^2 after the Euler step v + dt F (v = 0 after a restart)
  double vv = s.restart ? (s.dt * s.dt) * FF : VV + 2.0 * s.dt * P + (s.dt * s.dt) * FF;
  if (vv < 0.0) vv = 0.0;
  if (FF > 0.0) {
    s.cv = 1.0 - s.alpha;
    s.cf = s.alpha * sqrt(vv) / sqrt(FF);
  } else {
    s.cv = 1.0;
    s.cf = 0.0;
  }
  s.it += 1;
  if (s.it >= f.max_iter) {
    s.pending = 1;
    s.phase = PH_ENERGY;  // energy at these positions, then the last step
  }
  return;
}

// ---------------------------------------------------------------------------
// Force kernel: one atom per thread, 256 atoms of one slot per block.  Also
// the per-block partials (E, |F|^2, F.v, |v|^2, max |F_i|^2, W_xy, non-finite)
// and, in the last block of each slot, the FIRE control.

// Force of one atom li of the tile (TPA lanes), accumulated into the
// thread's partials: E, |F|^2, F.v, |v|^2 (conjugate gradients: F.F0, F0 the
// force at the line-search origin), max |F_i|^2, W_xy, non-finite, max |v_i|^2.
template <int D, bool WE, int TPA, bool LDS>
__device__ __forceinline__ void force_atom(const IterArgs& a, const Geom& g, int li, int col,
                                           const double (*sh)[4], const PairParams* spp,
                                           const double* hx, const double* hy, const double* hz,
                                           bool cg, double* part) {
  const int64_t gi = g.atom_off + li;
  const double4 pi = a.pos4[gi];
  double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0, w = 0.0;
  if (LDS)
    atom_pairs_packed<D, WE, TPA>(pi, (int)pi.w, a.nbp + g.nb_off / kGroup, col, g.npad,
                                  a.nbc[g.atom_off + col], a.max_nb, hx, hy, hz, spp, fx, fy, fz,
                                  e, w);
  else
    atom_pairs<D, WE, TPA>(pi, (int)pi.w, a.nbl + g.nb_off, col, g.npad, a.nbc[g.atom_off + col],
                           a.max_nb, (uint32_t)li | (13u << kCodeShift), a.pos4 + g.atom_off, sh,
                           spp, fx, fy, fz, e, w);
  if (threadIdx.x % TPA != 0) return;
  a.fx[gi] = fx;
  a.fy[gi] = fy;
  if (D == 3) a.fz[gi] = fz;
  const double vx = a.vx[gi], vy = a.vy[gi], vz = (D == 3) ? a.vz[gi] : 0.0;
  const double ff = fx * fx + fy * fy + fz * fz;
  const double vv = vx * vx + vy * vy + vz * vz;
  part[0] += 0.5 * e;
  part[1] += ff;
  part[2] += fx * vx + fy * vy + fz * vz;
  if (cg)
    part[3] += fx * a.gx[gi] + fy * a.gy[gi] + ((D == 3) ? fz * a.gz[gi] : 0.0);
  else
    part[3] += vv;
  part[4] = fmax(part[4], ff);
  part[5] += 0.5 * w;
  if (!(isfinite(e) && isfinite(ff) && isfinite(pi.x + pi.y + pi.z))) part[6] = 1.0;
  part[7] = fmax(part[7], vv);
}

template <int D, bool WE, int TPA, bool LDS>
__device__ __forceinline__ void force_tile(const IterArgs& a, const Geom& g, int a0, int a1,
                                           const double (*sh)[4], const PairParams* spp,
                                           const double* hx, const double* hy, const double* hz,
                                           bool cg, double* part) {
  constexpr int per = kBlock / TPA;
  for (int b = a0; b < a1; b += per) {
    const int k = b + (int)(threadIdx.x / TPA);
    if (k < a1)
      force_atom<D, WE, TPA, LDS>(a, g, a.tord[g.atom_off + k], k, sh, spp, hx, hy, hz, cg, part);
  }
}

// Force kernel: one block per force tile (a segment of a cell row, tiles.h).
// Sized for five wavefronts per SIMD: at most 96 VGPRs (pairs walked two at
// a time) and under 32 KB of LDS per block (the compact halo capacity).
// The block reads the tile's header and halo run table, stages the halo into
// LDS (image shifts applied), then TPA lanes per atom walk each neighbour
// list.  Writes F and the tile partials (force_atom); k_control combines
// them.
// The critical chain of a live round shares compute units with the batch:
// its waves take the highest issue priority of their SIMD.
__device__ __forceinline__ void critical_priority(const IterArgs& a) {
  if (a.prio) __builtin_amdgcn_s_setprio(3);
}

template <int D, int TPA, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(W))) void k_force(IterArgs a) {
  critical_priority(a);
  // (slot, global tile index): computed for a lane of one slot, else read in one load
  int2 bt;
  if (a.one_rep >= 0) {
    const int t = one_slot_item(blockIdx.x, a.one_ntiles);
    bt = make_int2(t < 0 ? -1 : a.one_rep, a.one_tile0 + t);
  } else {
    const uint64_t ent = reinterpret_cast<const uint64_t*>(a.ftiles)[blockIdx.x];
    bt = make_int2((int)(uint32_t)ent, (int)(uint32_t)(ent >> 32));
  }
  const int rep = bt.x;
  if (rep < 0) return;
  const int tid = threadIdx.x;
  constexpr int CAP = (D == 3) ? kHaloCap3 : kHaloCap2;
  constexpr int SU = (CAP + kBlock - 1) / kBlock;
  // The tile header and this thread's compact-halo indices (only the halo's
  // own entries: reading the whole capacity ahead of the header cost 5 % more
  // fetched bytes and gained no time), with the slot's state and geometry in
  // flight meanwhile.
  const int64_t tix = bt.y;
  const TileHdr hdr = reinterpret_cast<const TileHdr*>(a.thdr)[tix];
  uint32_t hent[SU];
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int h = tid + u * kBlock;
    hent[u] = h < hdr.halo ? a.hidx[tix * CAP + h] : 0u;
  }
  const State* stp = a.state + rep;
  const int phase = stp->phase;
  const int ntiles = stp->ntiles;
  const Geom g = a.geom[rep];
  const bool we = phase_energy(phase);
  const bool compute = phase_force(phase);
  if (!compute || tix - g.tile_off >= ntiles) return;
  const bool cg = (phase == PH_CG);

  __shared__ double hx[CAP];
  __shared__ double hy[CAP];
  __shared__ double hz[D == 3 ? CAP : 1];
  __shared__ double sh[32][4];
  __shared__ PairParams spp[4];
  __shared__ double red[kForceParts][kBlock / kWave];
  constexpr int ops[kForceParts] = {0, 0, 0, 0, 1, 0, 1, 1};

  double part[kForceParts] = {0, 0, 0, 0, 0, 0, 0, 0};
  {
    const Box bx = box_at(g, stp->k);
    if (tid >= 32 && tid < 32 + 27) code_shift(tid - 32, bx, sh[tid - 32]);
    if (tid >= 64 && tid < 68) spp[tid - 64] = a.pp[tid - 64];
    __syncthreads();
    if (hdr.halo >= 0) {
      stage_halo_from<D, CAP>(hdr, hent, sh, a.pos4 + g.atom_off, hx, hy, hz);
      if (tid == kBlock - 1) {   // the far fill slot (the builder keeps halos below CAP)
        hx[CAP - 1] = kFarFill;
        hy[CAP - 1] = kFarFill;
        if (D == 3) hz[CAP - 1] = kFarFill;
      }
      __syncthreads();
      if (we)
        force_tile<D, true, TPA, true>(a, g, hdr.a0, hdr.a1, sh, spp, hx, hy, hz, cg, part);
      else
        force_tile<D, false, TPA, true>(a, g, hdr.a0, hdr.a1, sh, spp, hx, hy, hz, cg, part);
    } else {
      if (we)
        force_tile<D, true, TPA, false>(a, g, hdr.a0, hdr.a1, sh, spp, hx, hy, hz, cg, part);
      else
        force_tile<D, false, TPA, false>(a, g, hdr.a0, hdr.a1, sh, spp, hx, hy, hz, cg, part);
    }
    block_reduce<kForceParts>(part, ops, red);
    if (tid == 0) {
      double* dst = a.fpart + tix * kForceParts;
#pragma unroll
      for (int c = 0; c < kForceParts; ++c) dst[c] = part[c];
    }
  }
}

// The slot's sums of one iteration: each thread's share of the force
// tiles' partials (E, |F|^2, F.v, |v|^2, max |F_i|^2, W_xy, non-finite, max
// |d_i|^2 in r[8]) and of the update's max displacements (r[7], from upart),
// in tile order; slot_reduce then combines the threads by a fixed tree
// (result in thread 0).  The kernel boundary after the force kernel makes
// the partials visible; no device-scope fences inside the force kernel.
__device__ __forceinline__ void slot_partials(const IterArgs& a, const Geom& g, int ntiles,
                                              bool compute, double* r) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int c = 0; c < kForceParts + 1; ++c) r[c] = 0.0;
  if (compute) {
    for (int b = tid; b < ntiles; b += kBlock) {
      const double* src = a.fpart + ((int64_t)g.tile_off + b) * kForceParts;
      r[0] += src[0];
      r[1] += src[1];
      r[2] += src[2];
      r[3] += src[3];
      r[4] = fmax(r[4], src[4]);
      r[5] += src[5];
      r[6] = fmax(r[6], src[6]);
      r[8] = fmax(r[8], src[7]);
    }
    for (int b = tid; b < g.nblocks; b += kBlock) r[7] = fmax(r[7], a.upart[g.block0 + b]);
  }
}

__device__ __forceinline__ void slot_reduce(double* r, double (*red)[kBlock / kWave]) {
  constexpr int ops[kForceParts + 1] = {0, 0, 0, 0, 1, 0, 1, 1, 1};
  block_reduce<kForceParts + 1>(r, ops, red);
}

// Control alone, one block per slot of the selection, the state updated in
// place: the single force evaluation of aqs_energy_forces (PH_EVAL).
template <bool CG>
__global__ __launch_bounds__(kBlock) void k_control(IterArgs a) {
  const int rep = a.sel[blockIdx.x];
  const State* stp = a.state + rep;
  const int tid = threadIdx.x;
  State s0;
  if (tid == 0) copy_state(s0, *stp);
  const int phase = stp->phase;
  const bool compute = phase_force(phase);
  const bool counted = compute || phase == PH_FINISH || phase == PH_STOP;
  if (!counted) return;
  const Geom g = a.geom[rep];
  __shared__ double red[kForceParts + 1][kBlock / kWave];
  double r[kForceParts + 1];
  slot_partials(a, g, stp->ntiles, compute, r);
  slot_reduce(r, red);
  if (tid == 0) {
    if (compute) atomicAdd(a.evals, (unsigned long long)g.n);
    CgState q;
    if (CG) q = a.cgst[rep];
    control<CG>(a, rep, g, r, phase, s0, q, true);
    copy_state(a.state[rep], s0);
    if (CG) a.cgst[rep] = q;
  }
}

// ---------------------------------------------------------------------------
// One iteration's control and move, after the force kernel.  Every block of
// a slot sums the slot's tile partials and runs the control on them (the same
// fixed-order sums, so every block reaches the same new state), then applies
// to its 256 atoms the FIRE update (steps 5-9 of the minimiser), the
// conjugate-gradient move, the fine affine step of the chain or the learned
// start's move, and records its max |u_i| = |r_i - F x_ref,i| for the list
// test.  State, conjugate-gradient state and displacement partials are
// double-buffered: the blocks read a.state, a.cgst and a.upart and write
// a.state_out, a.cgst_out (block 0 of the slot) and a.upart_out, and the host
// swaps the two buffers from one iteration to the next, so no block reads
// what another block of the same launch writes.  Every block of the table
// writes its outputs, also when its slot is idle, so the out buffers always
// hold the latest values.  The states pass through LDS one dword per thread
// (the control, in thread 0, works on the LDS copy), which keeps the kernel's
// registers, and so its blocks per CU, for the batch.  PF: the atoms' data
// are loaded before the control (a lane of one slot, latency-bound); without
// it they are loaded after it, with fewer registers held meanwhile.
constexpr int kStateWords = (int)(sizeof(State) / 4);
constexpr int kCgWords = (int)(sizeof(CgState) / 4);
static_assert(sizeof(State) % 4 == 0 && sizeof(CgState) % 4 == 0 && kStateWords <= kBlock &&
                  kCgWords <= kBlock, "states move as dwords, one per thread");

template <int D, bool CG, bool PF>
__global__ __launch_bounds__(kBlock) void k_step(IterArgs a) {
  critical_priority(a);
  int2 bt;
  if (a.one_rep >= 0) {
    const int b = one_slot_item(blockIdx.x, a.one_nblk);
    bt = make_int2(b < 0 ? -1 : a.one_rep, b);
  } else {
    bt = a.blocks[blockIdx.x];
  }
  const int rep = bt.x;
  if (rep < 0) return;
  const int tid = threadIdx.x;
  const bool owner = (bt.y == 0);
  const State* sin = a.state + rep;
  // this thread's dwords of the slot's state and conjugate-gradient state
  uint32_t sw = 0u, qw = 0u;
  if (tid < kStateWords) sw = reinterpret_cast<const uint32_t*>(sin)[tid];
  if (CG && tid < kCgWords) qw = reinterpret_cast<const uint32_t*>(a.cgst + rep)[tid];
  const int phase0 = sin->phase;
  const int ntiles = sin->ntiles;
  const Geom g = a.geom[rep];
  const int ub = g.block0 + bt.y;
  const bool compute = phase_force(phase0);
  const bool counted = compute || phase0 == PH_FINISH || phase0 == PH_STOP;
  if (!counted) {
    // nothing to control or move: carry the slot over to the out buffers
    if (tid == 0) a.upart_out[ub] = a.upart[ub];
    if (owner) {
      if (tid < kStateWords) reinterpret_cast<uint32_t*>(a.state_out + rep)[tid] = sw;
      if (CG && tid < kCgWords) reinterpret_cast<uint32_t*>(a.cgst_out + rep)[tid] = qw;
    }
    return;
  }
  const int li = bt.y * kBlock + tid;
  const bool mine = li < g.n;
  const int64_t gi = g.atom_off + li;
  // this thread's atom, in flight while the control runs
  double4 p = make_double4(0.0, 0.0, 0.0, 0.0), x0 = p;
  double vx = 0.0, vy = 0.0, vz = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
  auto load_atom = [&]() {
    if (mine) {
      p = a.pos4[gi];
      x0 = a.xref4[gi];
      vx = a.vx[gi];
      vy = a.vy[gi];
      if (D == 3) vz = a.vz[gi];
      fx = a.fx[gi];
      fy = a.fy[gi];
      if (D == 3) fz = a.fz[gi];
    }
  };
  if (PF) load_atom();
  __shared__ double red[kForceParts + 1][kBlock / kWave];
  __shared__ State ss;
  __shared__ CgState sq;
  {
    double r[kForceParts + 1];
    slot_partials(a, g, ntiles, compute, r);
    if (tid < kStateWords) reinterpret_cast<uint32_t*>(&ss)[tid] = sw;
    if (CG && tid < kCgWords) reinterpret_cast<uint32_t*>(&sq)[tid] = qw;
    slot_reduce(r, red);   // its barriers also publish ss and sq
    if (tid == 0) {
      if (owner && compute) {
        atomicAdd(a.evals, (unsigned long long)g.n);
        if (a.tevals) atomicAdd(a.tevals, (unsigned long long)g.n);
      }
      control<CG>(a, rep, g, r, phase0, ss, sq, owner);
    }
    __syncthreads();
  }
  if (owner) {
    if (tid < kStateWords)
      reinterpret_cast<uint32_t*>(a.state_out + rep)[tid] = reinterpret_cast<const uint32_t*>(&ss)[tid];
    if (CG && tid < kCgWords)
      reinterpret_cast<uint32_t*>(a.cgst_out + rep)[tid] = reinterpret_cast<const uint32_t*>(&sq)[tid];
  }
  if (!PF) load_atom();
  const int phase = ss.phase;
  const bool fire = !CG && (phase == PH_FIRE || phase == PH_STOP);
  const bool cg = CG && (phase == PH_CG || phase == PH_STOP);
  const bool adv = (phase == PH_ADVANCE);
  // learned start: move to F r + dgamma (u_hat - mean u_hat), or back
  const bool lmove = (phase == PH_LMOVE || phase == PH_LREVERT);
  const bool moves = fire || cg || adv || lmove;
  if (!moves) {
    // no move: the displacement since the build is unchanged
    if (tid == 0) a.upart_out[ub] = a.upart[ub];
    if (phase != PH_FINISH) return;
  }
  double m[1] = {0.0};
  if (mine) {
    if (ss.do_snap && (adv || phase == PH_FINISH)) {  // first inherent structure -> snap_dst
      const Geom gd = a.geom[ss.snap_dst];
      const int64_t di = gd.atom_off + li;
      a.pos4[di] = p;
      const int32_t aid = a.id[gi];
      a.id[di] = aid;
      a.inv[gd.atom_off + aid] = li;
    }
    if (fire) {
      const double dt = ss.dt, cv = ss.cv, cf = ss.cf, dmax = a.fire.dmax;
      if (ss.restart) {
        p.x -= 0.5 * dt * vx;
        p.y -= 0.5 * dt * vy;
        if (D == 3) p.z -= 0.5 * dt * vz;
        vx = 0.0;
        vy = 0.0;
        vz = 0.0;
      }
      vx += dt * fx;
      vy += dt * fy;
      vz += dt * fz;
      vx = cv * vx + cf * fx;
      vy = cv * vy + cf * fy;
      vz = cv * vz + cf * fz;
      const double sp = dt * sqrt(vx * vx + vy * vy + vz * vz);
      if (sp > dmax) {
        const double sc = dmax / sp;
        vx *= sc;
        vy *= sc;
        vz *= sc;
      }
      p.x += dt * vx;
      p.y += dt * vy;
      if (D == 3) p.z += dt * vz;
      a.pos4[gi] = p;
      a.vx[gi] = vx;
      a.vy[gi] = vy;
      if (D == 3) a.vz[gi] = vz;
    } else if (cg) {
      // conjugate gradients: d lives in v; a new direction also saves F0
      double dx = vx, dy = vy, dz = vz;
      if (sq.newdir) {
        const double b = sq.beta;
        if (b == 0.0) {
          dx = fx;
          dy = fy;
          dz = fz;
        } else {
          dx = fx + b * dx;
          dy = fy + b * dy;
          dz = fz + b * dz;
        }
        a.gx[gi] = fx;
        a.gy[gi] = fy;
        if (D == 3) a.gz[gi] = fz;
        a.vx[gi] = dx;
        a.vy[gi] = dy;
        if (D == 3) a.vz[gi] = dz;
      }
      const double da = sq.step;
      p.x += da * dx;
      p.y += da * dy;
      if (D == 3) p.z += da * dz;
      a.pos4[gi] = p;
    } else if (adv) {
      if (g.dgamma_y == 0.0) {
        // Eq. (16): x <- x + dgamma y, written out (no fused multiply-add), as
        // the learned start's plain move does, so both give the same bits
#pragma clang fp contract(off)
        p.x += g.dgamma * p.y;
      } else {
        // Eq. (17): (x, y) <- F (x, y), both from the old coordinates
#pragma clang fp contract(off)
        const double x = p.x, y = p.y;
        p.x = x + g.dgamma * y;
        p.y = g.dgamma_y * x + y;
      }
      a.pos4[gi] = p;
      a.vx[gi] = 0.0;
      a.vy[gi] = 0.0;
      if (D == 3) a.vz[gi] = 0.0;
    } else if (lmove) {
      // dl holds u_hat per unit strain (network, extrapolation), or the
      // displacement itself (linear response, lmean = 0: exactly x0 + u)
      const double sc = (ss.start_mode == kStartLinear) ? 1.0 : g.dgamma;
      const double ux = sc * (a.dlx[gi] - ss.lmean[0]);
      const double uy = sc * (a.dly[gi] - ss.lmean[1]);
      const double uz = (D == 3) ? sc * (a.dlz[gi] - ss.lmean[2]) : 0.0;
      if (phase == PH_LMOVE) {
        p.x += ux;
        p.y += uy;
        if (D == 3) p.z += uz;
      } else {
        const double4 q = a.alt4[gi];   // the plain start, bit for bit
        p.x = q.x;
        p.y = q.y;
        p.z = q.z;
      }
      a.pos4[gi] = p;
    }
    if (moves) {
      // written out, as in the learned start's plain move: both paths take
      // the same list-rebuild decisions bit for bit
#pragma clang fp contract(off)
      double ux, uy;
      if (g.dgamma_y == 0.0) {
        const double gd = strain_of(ss.k, g.dgamma) - ss.gamma_build;
        ux = p.x - (x0.x + gd * x0.y);
        uy = p.y - x0.y;
      } else {
        double G[4];
        strain_since(g, ss.k, ss.k_build, G);
        ux = p.x - (G[0] * x0.x + G[1] * x0.y);
        uy = p.y - (G[2] * x0.x + G[3] * x0.y);
      }
      const double uz = p.z - x0.z;
      m[0] = sqrt(ux * ux + uy * uy + uz * uz);
    }
  }
  if (moves) {
    const int op[1] = {1};
    block_reduce<1>(m, op, red);
    if (tid == 0) a.upart_out[ub] = m[0];
  }
}

// A launch, timed by the runtime from the kernel's start to its end when
// events are given (hipExtLaunchKernelGGL records them with the dispatch
// itself: no marker packets between the kernels, and no dispatch gap in the
// interval).
template <typename K>
void launch_timed(K kernel, int32_t grid, int32_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                  const IterArgs& a) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), (uint32_t)lds, s, e0, e1, 0u, a);
  else
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), lds, s, a);
}

template <int D, int TPA>
void launch_force_t(const IterArgs& a, int32_t ntiles, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.waves == 4)
    launch_timed(k_force<D, TPA, 4>, ntiles, a.lds_pad, s, e0, e1, a);
  else
    launch_timed(k_force<D, TPA, 5>, ntiles, a.lds_pad, s, e0, e1, a);
}

template <int D>
void launch_force_d(const IterArgs& a, int32_t ntiles, int32_t tpa, hipStream_t s, hipEvent_t e0,
                    hipEvent_t e1) {
  switch (tpa) {
    case 1: launch_force_t<D, 1>(a, ntiles, s, e0, e1); break;
    case 2: launch_force_t<D, 2>(a, ntiles, s, e0, e1); break;
    case 4: launch_force_t<D, 4>(a, ntiles, s, e0, e1); break;
    default: launch_force_t<D, 8>(a, ntiles, s, e0, e1); break;
  }
}

// Dynamic LDS to add to each force block so that at most `blocks` of them
// fit on a CU and one more block of the same kernel still does: with static
// LDS S per block and LDS C per CU, the padded size X satisfies
// (blocks + 1) X > C and blocks X + S <= C.  0 if no such X exists.
template <int D, int TPA>
int32_t force_pad_d(int32_t blocks) {
  hipFuncAttributes fa{};
  int dev = 0, cu_lds = 0;
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_force<D, TPA, 5>)) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
          hipSuccess)
    return 0;
  const int64_t S = (int64_t)fa.sharedSizeBytes, C = cu_lds;
  const int64_t lo = C / (blocks + 1) + 1;              // smallest X with (blocks + 1) X > C
  const int64_t hi = (C - S) / blocks;                  // largest X with blocks X + S <= C
  if (blocks < 1 || lo > hi || lo <= S) return 0;
  const int64_t X = std::min(hi, (lo + 511) / 512 * 512);  // a 512-byte multiple when one fits
  return (int32_t)(X - S);
}

int32_t force_lds_pad(int32_t dim, int32_t tpa, int32_t blocks) {
  if (dim == 3) {
    switch (tpa) {
      case 1: return force_pad_d<3, 1>(blocks);
      case 2: return force_pad_d<3, 2>(blocks);
      case 4: return force_pad_d<3, 4>(blocks);
      default: return force_pad_d<3, 8>(blocks);
    }
  }
  switch (tpa) {
    case 1: return force_pad_d<2, 1>(blocks);
    case 2: return force_pad_d<2, 2>(blocks);
    case 4: return force_pad_d<2, 4>(blocks);
    default: return force_pad_d<2, 8>(blocks);
  }
}

void launch_force(const IterArgs& a, int32_t ntiles, int32_t dim, hipStream_t s, hipEvent_t e0,
                  hipEvent_t e1) {
  if (ntiles <= 0) return;
  if (dim == 3)
    launch_force_d<3>(a, ntiles, a.tpa, s, e0, e1);
  else
    launch_force_d<2>(a, ntiles, a.tpa, s, e0, e1);
}

void launch_control(const IterArgs& a, hipStream_t s) {
  if (a.minimizer == kMinCG)
    hipLaunchKernelGGL(k_control<true>, dim3(a.nsel), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_control<false>, dim3(a.nsel), dim3(kBlock), 0, s, a);
}

template <int D, bool CG>
void launch_step_d(const IterArgs& a, int32_t nblk, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  // a lane of one slot is latency-bound: its atoms' data load during the control
  if (a.one_rep >= 0)
    launch_timed(k_step<D, CG, true>, nblk, 0, s, e0, e1, a);
  else
    launch_timed(k_step<D, CG, false>, nblk, 0, s, e0, e1, a);
}

void launch_step(const IterArgs& a, int32_t nblk, int32_t dim, hipStream_t s, hipEvent_t e0,
                 hipEvent_t e1) {
  if (nblk <= 0) return;
  const bool cg = (a.minimizer == kMinCG);
  if (dim == 3) {
    if (cg)
      launch_step_d<3, true>(a, nblk, s, e0, e1);
    else
      launch_step_d<3, false>(a, nblk, s, e0, e1);
  } else {
    if (cg)
      launch_step_d<2, true>(a, nblk, s, e0, e1);
    else
      launch_step_d<2, false>(a, nblk, s, e0, e1);
  }
}


// ---------------------------------------------------------------------------
// Affine simple shear of whole slots, Eqs. (2)-(3) with Eq. (16):
// x <- x + dg_r y, dg_r = dk_r dgamma_r formed on the host in one product.

__global__ __launch_bounds__(kBlock) void k_affine(const int2* blocks, const Geom* geom,
                                                    double4* pos4, const double* dg) {
  const int2 bt = blocks[blockIdx.x];
  if (bt.x < 0) return;
  const Geom& g = geom[bt.x];
  const int li = bt.y * kBlock + threadIdx.x;
  if (li >= g.n) return;
  double4 p = pos4[g.atom_off + li];
  const double* M = dg + 4 * (int64_t)bt.x;
  if (g.dgamma_y == 0.0) {
    p.x += M[1] * p.y;
  } else {
    // the pure shear's F^dk (Eq. 17), formed on the host
#pragma clang fp contract(off)
    const double x = p.x, y = p.y;
    p.x = M[0] * x + M[1] * y;
    p.y = M[2] * x + M[3] * y;
  }
  pos4[g.atom_off + li] = p;
}

void launch_affine(const int2* blocks, int32_t nblk, const Geom* geom, double4* pos4,
                   const double* dg_per_slot, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(k_affine, dim3(nblk), dim3(kBlock), 0, s, blocks, geom, pos4, dg_per_slot);
}

__global__ __launch_bounds__(kBlock) void k_reset_iter(const int2* blocks, const Geom* geom,
                                                        double* vx, double* vy, double* vz,
                                                        double* upart, int dim) {
  const int2 bt = blocks[blockIdx.x];
  if (bt.x < 0) return;
  const Geom& g = geom[bt.x];
  const int li = bt.y * kBlock + threadIdx.x;
  if (threadIdx.x == 0) upart[g.block0 + bt.y] = 0.0;
  if (li >= g.n) return;
  const int64_t gi = g.atom_off + li;
  vx[gi] = 0.0;
  vy[gi] = 0.0;
  if (dim == 3) vz[gi] = 0.0;
}

void launch_reset_iter(const int2* blocks, int32_t nblk, const Geom* geom, double* vx,
                       double* vy, double* vz, double* upart, int32_t dim, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(k_reset_iter, dim3(nblk), dim3(kBlock), 0, s, blocks, geom, vx, vy, vz,
                     upart, dim);
}

__global__ __launch_bounds__(kBlock) void k_copy_slot(const Geom* geom, int src, int dst, int n,
                                                       double4* pos4, int32_t* id,
                                                       int32_t* inv) {
  const int li = blockIdx.x * kBlock + threadIdx.x;
  if (li >= n) return;
  const int64_t so = geom[src].atom_off, d0 = geom[dst].atom_off;
  pos4[d0 + li] = pos4[so + li];
  id[d0 + li] = id[so + li];
  inv[d0 + li] = inv[so + li];
}

void launch_copy_slot(const Geom* geom, int32_t src, int32_t dst, int32_t n, double4* pos4,
                      int32_t* id, int32_t* inv, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy_slot, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, geom, src,
                     dst, n, pos4, id, inv);
}

// ---------------------------------------------------------------------------
// Distance of the equality test (Eq. 20): per atom id, the minimum image of
// r_a - r_b in the box of slot a; per-block maximum.

template <int D>
__global__ __launch_bounds__(kBlock) void k_compare(const Geom* geom, int ra, int rb, int n,
                                                     const double4* pos4, const int32_t* inv,
                                                     Box bx, double* part) {
  __shared__ double red[kForceParts][kBlock / kWave];
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  double m[1] = {0.0};
  if (idx < n) {
    const Geom& ga = geom[ra];
    const Geom& gb = geom[rb];
    const double4 pa = pos4[ga.atom_off + inv[ga.atom_off + idx]];
    const double4 pb = pos4[gb.atom_off + inv[gb.atom_off + idx]];
    double dx = pa.x - pb.x, dy = pa.y - pb.y, dz = (D == 3) ? pa.z - pb.z : 0.0;
    // fractional coordinates, nearest integer, back (Sec. 2.1 periodicity)
    double sf[3];
    frac(bx, dx, dy, dz, sf);
    double sx = sf[0], sy = sf[1], sz = (D == 3) ? sf[2] : 0.0;
    sx -= rint(sx);
    sy -= rint(sy);
    sz -= rint(sz);
    if (bx.h10 == 0.0) {
      dx = bx.h00 * sx + bx.h01 * sy;
      dy = bx.h11 * sy;
    } else {
      dx = bx.h00 * sx + bx.h01 * sy;
      dy = bx.h10 * sx + bx.h11 * sy;
    }
    dz = bx.h22 * sz;
    m[0] = sqrt(dx * dx + dy * dy + dz * dz);
  }
  const int op[1] = {1};
  block_reduce<1>(m, op, red);
  if (threadIdx.x == 0) part[blockIdx.x] = m[0];
}

void launch_compare(const Geom* geom, int32_t ra, int32_t rb, int32_t n, const double4* pos4,
                    const int32_t* inv, const Box& box, int32_t dim, double* part, hipStream_t s) {
  const int nb = (n + kBlock - 1) / kBlock;
  if (nb <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_compare<3>, dim3(nb), dim3(kBlock), 0, s, geom, ra, rb, n, pos4, inv, box,
                       part);
  else
    hipLaunchKernelGGL(k_compare<2>, dim3(nb), dim3(kBlock), 0, s, geom, ra, rb, n, pos4, inv, box,
                       part);
}

// ---------------------------------------------------------------------------
// Energy and virial W_ab = sum_{i<j} U'(r) d_a d_b / r of one slot, from the
// neighbour list; per block: E then W row-major 3x3.

template <int D>
__global__ __launch_bounds__(kBlock) void k_virial(IterArgs a, int rep, Box bx, double* part) {
  __shared__ double sh[27][4];
  __shared__ PairParams spp[4];
  __shared__ double red[kForceParts][kBlock / kWave];
  const Geom g = a.geom[rep];
  const int tid = threadIdx.x;
  if (tid < 27) code_shift(tid, bx, sh[tid]);
  if (tid < 4) spp[tid] = a.pp[tid];
  __syncthreads();
  const int col = blockIdx.x * kBlock + tid;   // list column (the tiles' walk order)
  double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (col < g.n) {
    const int li = a.tord[g.atom_off + col];
    const int64_t gi = g.atom_off + li;
    const double4 pi = a.pos4[gi];
    const int ti = (int)pi.w;
    const uint32_t* L = a.nbl + g.nb_off + col;
    const double4* P = a.pos4 + g.atom_off;
    const int32_t counts = a.nbc[g.atom_off + col];
    const int na = counts & 0xffff, nb = (counts >> 16) & 0xffff;
    for (int kk = 0; kk < na + nb; ++kk) {
      const int k = kk < na ? kk : a.max_nb - 1 - (kk - na);   // A rows, then B rows
      const uint32_t ent = L[(int64_t)k * g.npad];
      const double4 pj = P[ent & kIdxMask];
      const int code = (int)((ent >> kCodeShift) & 31u);
      double d[3];
      d[0] = (pj.x - pi.x) + sh[code][0];
      d[1] = (pj.y - pi.y) + sh[code][1];
      d[2] = (D == 3) ? (pj.z - pi.z) + sh[code][2] : 0.0;
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const PairParams q = spp[2 * ti + (kk < na ? 0 : 1)];
      if (r2 < q.rc2) {
        const double inv = recip_nr(r2);
        const double s2 = q.sig2 * inv;
        const double s6 = s2 * s2 * s2;
        const double s12 = s6 * s6;
        v[0] += 0.5 * (q.eps4 * (s12 - s6) - q.ucut);
        const double gg = q.eps4 * (6.0 * s6 - 12.0 * s12) * inv;
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
          for (int y = 0; y < 3; ++y) v[1 + 3 * x + y] += 0.5 * gg * d[x] * d[y];
      }
    }
  }
  // two passes of 5 values through the 8-wide reduction buffer
  const int op[5] = {0, 0, 0, 0, 0};
  double lo[5] = {v[0], v[1], v[2], v[3], v[4]};
  double hi[5] = {v[5], v[6], v[7], v[8], v[9]};
  block_reduce<5>(lo, op, red);
  block_reduce<5>(hi, op, red);
  if (tid == 0) {
    double* dst = part + (int64_t)blockIdx.x * 10;
    for (int c = 0; c < 5; ++c) {
      dst[c] = lo[c];
      dst[5 + c] = hi[c];
    }
  }
}

void launch_virial(const IterArgs& a, int32_t rep, int32_t nblocks, int32_t dim, const Box& box,
                   double* part, hipStream_t s) {
  if (nblocks <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_virial<3>, dim3(nblocks), dim3(kBlock), 0, s, a, rep, box, part);
  else
    hipLaunchKernelGGL(k_virial<2>, dim3(nblocks), dim3(kBlock), 0, s, a, rep, box, part);
}

}  // namespace aqs
