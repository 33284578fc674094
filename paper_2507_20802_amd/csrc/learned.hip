// learned.hip -- the learned start of an AQS step on gfx950: neighbourhood
// descriptors (FP64), the per-atom network 64 -> 128 -> 128 -> d on BF16
// matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), its training
// (fused forward/backward per 64 samples, fixed-order reduction, Adam), and
// the non-affine targets taken from plain AQS steps.
//
// The paper minimises from the affine start F r (Eq. 12); a better start for
// the minimiser is its outlook (Sec. 5).  The learned start is
// F r + dgamma (u_hat - mean u_hat), u_hat the predicted non-affine
// displacement per unit strain of each atom; the plain start stays the
// fallback (checks in k_lctl and in the control of the force iteration).
//
// Matrix-core tiles: a 16 x 16 FP32 tile D += A (16 x 32) B (32 x 16), BF16
// operands.  Lane l of the wavefront holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16] (j = 0..7) and receives D[4 (l / 16) + i][l % 16]
// (i = 0..3).  Operands are stored "k contiguous" so every fragment is one
// 16-byte load.
#include <hip/hip_runtime.h>
#include <algorithm>

#include "cellgeom.h"
#include "kernels.h"
#include "learned.h"
#include "tiles.h"

namespace aqs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even; NaN stays NaN.
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t b = __float_as_uint(x);
  if ((b & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float silu(float a) { return a / (1.0f + expf(-a)); }

__device__ __forceinline__ float dsilu(float a) {
  const float s = 1.0f / (1.0f + expf(-a));
  return s * (1.0f + a * (1.0f - s));
}

// Sum and max over a block of 256 threads in a fixed order.
template <int NV>
__device__ __forceinline__ void block_reduce_fixed(double* v, const int* op, double (*lds)[4]) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_xor(x, o, 64);
      x = op[k] ? fmax(x, y) : x + y;
    }
    if (lane == 0) lds[k][w] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double a = op[k] ? fmax(lds[k][0], lds[k][1]) : lds[k][0] + lds[k][1];
    const double b = op[k] ? fmax(lds[k][2], lds[k][3]) : lds[k][2] + lds[k][3];
    v[k] = op[k] ? fmax(a, b) : a + b;
  }
  __syncthreads();
}

constexpr double kMuLo = 0.6, kMuHi = 2.5;
// e^-(b - 1/2), b = 0..23 (entry 0 unused)
__constant__ double kGaussStep[24] = {
    1.6487212707001282, 0.6065306597126334, 0.22313016014842982, 0.0820849986238988,
    0.0301973834223185, 0.011108996538242306, 0.004086771438464067, 0.0015034391929775724,
    0.0005530843701478336, 0.00020346836901064417, 7.48518298877006e-05, 2.7536449349747158e-05,
    1.013009359863071e-05, 3.726653172078671e-06, 1.3709590863840845e-06, 5.04347662567888e-07,
    1.8553913626159784e-07, 6.82560337633487e-08, 2.510999155743982e-08, 9.237449661970594e-09,
    3.398267819495071e-09, 1.2501528663867426e-09, 4.5990553786523166e-10, 1.6918979226151304e-10};

// ---------------------------------------------------------------------------
// Descriptors, one block per force tile (tiles.h): the tile's halo is staged
// in LDS as for the force kernel and kLDescTPA lanes per atom walk its
// neighbour list (every pair within the pair cutoff r_d is in the list).
// Radial: species of j x 24 Gaussians exp(-(r - mu_b)^2 / (2 w^2)) f_c(r);
// angular: f_c(r) max(0, n_k . r_ij / r)^2; f_c(r) = (cos(pi r / r_d) + 1)/2.
// FP64 sums; the lanes' partial sums are combined by a fixed butterfly.
constexpr int kLDescTPA = 4;

template <int D>
__device__ __forceinline__ void desc_pair(double dx, double dy, double dz, int pt, int tj,
                                          const LearnArgs& a, double w, double* acc) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (!(r2 < a.rd2[pt])) return;
  const double r = sqrt(r2);
  const double fc = 0.5 * (cos(M_PI * r / a.rd[pt]) + 1.0);
  const double s1 = (tj == 1) ? 1.0 : 0.0, s0 = 1.0 - s1;
  // Gaussians by recurrence: with x = (r - mu_0) / w,
  // g_b / g_(b-1) = e^x e^-(b - 1/2), so two exponentials per pair
  const double x0 = (r - kMuLo) / w;
  const double ex = exp(x0);
  double gb = exp(-0.5 * (x0 * x0)) * fc;
  acc[0] += s0 * gb;
  acc[24] += s1 * gb;
#pragma unroll
  for (int b = 1; b < 24; ++b) {
    gb *= ex * kGaussStep[b];
    acc[b] += s0 * gb;
    acc[24 + b] += s1 * gb;
  }
  const double ux = dx / r, uy = dy / r, uz = (D == 3) ? dz / r : 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    double cth = ux * a.dirs[k][0] + uy * a.dirs[k][1];
    if (D == 3) cth += uz * a.dirs[k][2];
    cth = fmax(cth, 0.0);
    acc[48 + k] += fc * (cth * cth);
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_ldesc(LearnArgs a) {
  const int2 bt = a.ftiles[blockIdx.x];
  const int rep = bt.x;
  if (rep < 0) return;
  const State* st = a.state + rep;
  if (a.mode == 0 && st->phase != PH_LDESC) return;
  const Geom g = a.geom[rep];
  if (bt.y - g.tile_off >= st->ntiles) return;   // entries hold global tile indices
  const int tid = threadIdx.x;
  constexpr int CAP = (D == 3) ? kHaloCap3 : kHaloCap2;
  __shared__ double hx[CAP];
  __shared__ double hy[CAP];
  __shared__ double hz[D == 3 ? CAP : 1];
  __shared__ double sh[32][4];
  const int64_t tix = bt.y;
  const TileHdr hdr = reinterpret_cast<const TileHdr*>(a.thdr)[tix];
  const Box bx = box_at(g, st->k);
  if (tid >= 32 && tid < 32 + 27) code_shift(tid - 32, bx, sh[tid - 32]);
  __syncthreads();
  const double4* P = a.pos4 + g.atom_off;
  const bool lds = hdr.halo >= 0;
  if (lds) stage_halo<D, CAP>(hdr, a.hidx + tix * CAP, sh, P, hx, hy, hz);
  __syncthreads();
  const double w = (kMuHi - kMuLo) / 23.0;
  constexpr int per = kBlock / kLDescTPA;
  const int sub = tid % kLDescTPA;
  for (int b0 = hdr.a0; b0 < hdr.a1; b0 += per) {
    const int col = b0 + tid / kLDescTPA;      // list column (the tile's walk order)
    // every lane of the wavefront runs the loop; lanes past the tile do no pairs
    const bool live = col < hdr.a1;
    const int colc = live ? col : hdr.a0;
    const int lic = a.tord[g.atom_off + colc];
    const int64_t gi = g.atom_off + lic;
    const double4 pi = P[lic];
    const int ti = (int)pi.w;
    const int32_t counts = live ? a.nbc[g.atom_off + colc] : 0;
    const int na = counts & 0xffff, nbn = (counts >> 16) & 0xffff;
    const uint32_t* L = a.nbl + g.nb_off + colc;
    // packed list of the slot as 16-bit entries: group row q, column c,
    // entry i at (q npad + c) kGroup + i
    const uint16_t* Lp = reinterpret_cast<const uint16_t*>(a.nbp + g.nb_off / kGroup);
    const int G = a.max_nb / kGroup;
    double acc[kFeat];
#pragma unroll
    for (int f = 0; f < kFeat; ++f) acc[f] = 0.0;
    // A neighbours first (rows 0.. up), then B neighbours (rows from the top down)
    for (int kk = sub; kk < na + nbn; kk += kLDescTPA) {
      const int tj = kk < na ? 0 : 1;
      double dx, dy, dz;
      if (lds) {
        const int q = kk < na ? kk : kk - na;
        const int grow = kk < na ? q / kGroup : G - 1 - q / kGroup;
        const uint32_t off = Lp[((int64_t)grow * g.npad + colc) * kGroup + q % kGroup];
        const int h = (int)(off >> 3);   // entries are byte offsets 8 h
        dx = hx[h] - pi.x;
        dy = hy[h] - pi.y;
        dz = (D == 3) ? hz[h] - pi.z : 0.0;
      } else {
        const int k = kk < na ? kk : a.max_nb - 1 - (kk - na);
        const uint32_t ent = L[(int64_t)k * g.npad];
        const double4 pj = P[ent & kIdxMask];
        const int code = (int)((ent >> kCodeShift) & 31u);
        dx = (pj.x - pi.x) + sh[code][0];
        dy = (pj.y - pi.y) + sh[code][1];
        dz = (D == 3) ? (pj.z - pi.z) + sh[code][2] : 0.0;
      }
      desc_pair<D>(dx, dy, dz, 2 * ti + tj, tj, a, w, acc);
    }
#pragma unroll
    for (int f = 0; f < kFeat; ++f) {
#pragma unroll
      for (int off = 1; off < kLDescTPA; off <<= 1) acc[f] += __shfl_xor(acc[f], off, 64);
    }
    if (!live || sub != 0) continue;
    if (a.mode == 1) {
      float* o = a.out + (int64_t)a.id[gi] * kFeat;
#pragma unroll
      for (int f = 0; f < kFeat; ++f) o[f] = (float)acc[f];
    } else {
      uint16_t zz[kFeat];
#pragma unroll
      for (int f = 0; f < kFeat; ++f)
        zz[f] = f2bf(((float)acc[f] - a.mlp->fmean[f]) / a.mlp->fstd[f]);
      uint4* o = reinterpret_cast<uint4*>(a.zbuf + gi * kFeat);
#pragma unroll
      for (int q = 0; q < kFeat / 8; ++q) {
        uint4 v;
        v.x = zz[8 * q + 0] | ((uint32_t)zz[8 * q + 1] << 16);
        v.y = zz[8 * q + 2] | ((uint32_t)zz[8 * q + 3] << 16);
        v.z = zz[8 * q + 4] | ((uint32_t)zz[8 * q + 5] << 16);
        v.w = zz[8 * q + 6] | ((uint32_t)zz[8 * q + 7] << 16);
        o[q] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Network forward for 16 rows per wavefront.  Weights in LDS ([out][in]),
// z rows from global memory; h1 and h2 go through the wave's LDS buffers.
constexpr int kHS = kHid + 8;   // row stride of the activation buffers

__device__ __forceinline__ f32x4 zero4() {
  f32x4 z = {0.f, 0.f, 0.f, 0.f};
  return z;
}

// y (standardised units) for the 16 rows whose z rows start at zrow (row
// (l % 16) at zrow + (l % 16) * 64); returns the lane's 4 rows of column l % 16.
__device__ __forceinline__ f32x4 mlp16(const uint16_t* zrow, const uint16_t* sw1,
                                       const uint16_t* sw2, const uint16_t* sw3, const float* b1,
                                       const float* b2, uint16_t (*h1)[kHS], uint16_t (*h2)[kHS]) {
  const int l = threadIdx.x % 64;
  const int lr = l & 15, lk = 8 * (l >> 4);
  const bf16x8 z0 = ld8(zrow + lr * kFeat + lk), z1 = ld8(zrow + lr * kFeat + lk + 32);
  f32x4 acc[8];
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    const uint16_t* wb = sw1 + (nt * 16 + lr) * kFeat + lk;
    acc[nt] = mma(z0, ld8(wb), zero4());
    acc[nt] = mma(z1, ld8(wb + 32), acc[nt]);
  }
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    const int col = nt * 16 + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i) h1[4 * (l >> 4) + i][col] = f2bf(silu(acc[nt][i] + b1[col]));
  }
  __syncthreads();
  bf16x8 hA[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) hA[kk] = ld8(&h1[lr][kk * 32 + lk]);
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    acc[nt] = zero4();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      acc[nt] = mma(hA[kk], ld8(sw2 + (nt * 16 + lr) * kHid + kk * 32 + lk), acc[nt]);
  }
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    const int col = nt * 16 + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i) h2[4 * (l >> 4) + i][col] = f2bf(silu(acc[nt][i] + b2[col]));
  }
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) hA[kk] = ld8(&h2[lr][kk * 32 + lk]);
  f32x4 y = zero4();
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) y = mma(hA[kk], ld8(sw3 + lr * kHid + kk * 32 + lk), y);
  return y;
}

// Tail of a predicted start, per atom li of block bt of a slot in PH_LDESC:
// the predicted displacement per unit strain u into dl, block partials (sum
// u, max |u|^2, non-finite, max displacement since the list build), the
// snapshot of the inherent structure if pending, then the plain start
// x <- x + dgamma y with v = 0, also saved in alt4.  Every thread of the
// block calls it (live = atom exists).
template <int D>
__device__ void predicted_start(const LearnArgs& a, const State* st, const Geom& g, int2 bt,
                                int li, bool live, double ux, double uy, double uz,
                                double (*red)[4]) {
  double part[kLearnParts] = {0, 0, 0, 0, 0, 0};
  if (live) {
    const int64_t gi = g.atom_off + li;
    a.dlx[gi] = ux;
    a.dly[gi] = uy;
    if (D == 3) a.dlz[gi] = uz;
    part[0] = ux;
    part[1] = uy;
    part[2] = uz;
    const double uu = ux * ux + uy * uy + uz * uz;
    part[3] = uu;
    part[4] = isfinite(uu) ? 0.0 : 1.0;
    double4 p = a.pos4[gi];
    if (st->do_snap) {  // first inherent structure of the chain -> snap_dst
      const Geom gd = a.geom[st->snap_dst];
      const int64_t di = gd.atom_off + li;
      a.pos4[di] = p;
      const int32_t aid = a.id[gi];
      a.id[di] = aid;
      a.inv[gd.atom_off + aid] = li;
    }
    if (g.dgamma_y == 0.0) {
      // plain start, Eq. (16), written out as in the move kernel's fine step
#pragma clang fp contract(off)
      p.x += g.dgamma * p.y;
    } else {
      const double x = p.x, y = p.y;   // plain start under the pure shear of Eq. (17)
      p.x = x + g.dgamma * y;
      p.y = g.dgamma_y * x + y;
    }
    a.pos4[gi] = p;
    a.alt4[gi] = p;          // restored bit for bit if the predicted start is rejected
    a.vx[gi] = 0.0;
    a.vy[gi] = 0.0;
    if (D == 3) a.vz[gi] = 0.0;
    const double4 x0 = a.xref4[gi];
    // the displacement since the build, written out as in the move kernel
    {
#pragma clang fp contract(off)
      double dx, dy;
      if (g.dgamma_y == 0.0) {
        const double gdl = strain_of(st->k + 1, g.dgamma) - st->gamma_build;
        dx = p.x - (x0.x + gdl * x0.y);
        dy = p.y - x0.y;
      } else {
        double G[4];
        strain_since(g, st->k + 1, st->k_build, G);
        dx = p.x - (G[0] * x0.x + G[1] * x0.y);
        dy = p.y - (G[2] * x0.x + G[3] * x0.y);
      }
      const double dz = p.z - x0.z;
      part[5] = sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  const int ops[kLearnParts] = {0, 0, 0, 1, 1, 1};
  block_reduce_fixed<kLearnParts>(part, ops, red);
  if (threadIdx.x == 0) {
    double* dst = a.lpart + (int64_t)(g.block0 + bt.y) * kLearnParts;
    for (int k = 0; k < kLearnParts; ++k) dst[k] = part[k];
    a.upart[g.block0 + bt.y] = part[5];
  }
}

// Inference over a (slot, 256-atom block): 4 wavefronts x 4 groups of 16.
// mode 0 (engine, slots in PH_LDESC): u_hat into dl, block partials, the
// snapshot of the inherent structure if pending, then the plain start
// x <- x + dgamma y with v = 0 and the displacement bound of the list test.
// mode 1: u_hat into out[id * d + c].
template <int D>
__global__ __launch_bounds__(kBlock) void k_lmlp(LearnArgs a) {
  const int2 bt = a.blocks[blockIdx.x];
  if (bt.x < 0) return;
  const State* st = a.state + bt.x;
  if (a.mode == 0 && st->phase != PH_LDESC) return;
  const Geom g = a.geom[bt.x];
  const MlpDev* M = a.mlp;
  __shared__ __attribute__((aligned(16))) uint16_t sw1[kHid * kFeat];
  __shared__ __attribute__((aligned(16))) uint16_t sw2[kHid * kHid];
  __shared__ __attribute__((aligned(16))) uint16_t sw3[kOutPad * kHid];
  __shared__ __attribute__((aligned(16))) uint16_t hb1[4][16][kHS];
  __shared__ __attribute__((aligned(16))) uint16_t hb2[4][16][kHS];
  __shared__ float uo[kBlock][4];
  __shared__ float sb[2 * kHid + kOutPad + 8];
  __shared__ double red[kLearnParts][4];
  const int tid = threadIdx.x;
  {
    const uint4* s1 = reinterpret_cast<const uint4*>(M->w1t);
    const uint4* s2 = reinterpret_cast<const uint4*>(M->w2t);
    const uint4* s3 = reinterpret_cast<const uint4*>(M->w3t);
    for (int q = tid; q < kHid * kFeat / 8; q += kBlock) reinterpret_cast<uint4*>(sw1)[q] = s1[q];
    for (int q = tid; q < kHid * kHid / 8; q += kBlock) reinterpret_cast<uint4*>(sw2)[q] = s2[q];
    for (int q = tid; q < kOutPad * kHid / 8; q += kBlock) reinterpret_cast<uint4*>(sw3)[q] = s3[q];
    if (tid < kHid) {
      sb[tid] = M->b1[tid];
      sb[kHid + tid] = M->b2[tid];
    }
    if (tid < kOutPad) sb[2 * kHid + tid] = M->b3[tid];
    if (tid < 4) {
      sb[2 * kHid + kOutPad + tid] = M->tmean[tid];
      sb[2 * kHid + kOutPad + 4 + tid] = M->tstd[tid];
    }
  }
  __syncthreads();
  const int w = tid / 64, l = tid % 64;
  const int dim = M->dim;
  for (int q = 0; q < 4; ++q) {
    const int row0 = bt.y * kBlock + w * 64 + q * 16;
    const f32x4 y = mlp16(a.zbuf + (g.atom_off + row0) * kFeat, sw1, sw2, sw3, sb, sb + kHid,
                          hb1[w], hb2[w]);
    const int c = l & 15;
    if (c < 4) {
      const float b3 = sb[2 * kHid + c];
      const float tm = sb[2 * kHid + kOutPad + c], ts = sb[2 * kHid + kOutPad + 4 + c];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float yy = y[i] + b3;
        const float pr = yy * ts;
        uo[w * 64 + q * 16 + 4 * (l >> 4) + i][c] = pr + tm;
      }
    }
    __syncthreads();
  }
  const int li = bt.y * kBlock + tid;
  const bool live = li < g.n;
  const int64_t gi = g.atom_off + li;
  if (a.mode == 1) {
    if (live) {
      float* o = a.out + (int64_t)a.id[gi] * dim;
      for (int cc = 0; cc < dim; ++cc) o[cc] = uo[tid][cc];
    }
    return;
  }
  // one call site for every thread (the tail synchronises the block)
  const double ux = live ? (double)uo[tid][0] : 0.0, uy = live ? (double)uo[tid][1] : 0.0;
  const double uz = (live && D == 3) ? (double)uo[tid][2] : 0.0;
  predicted_start<D>(a, st, g, bt, li, live, ux, uy, uz, red);
}

// Extrapolated start (the extrapolation the paper's conclusion, Sec. 5,
// proposes to cut the minimiser's iterations): the non-affine displacement
// of the step just finished, u_(k-1) = r(IS_(k-1)) - F r(IS_(k-2)), per unit
// strain, predicts the next one.  alt4 still holds the plain start
// F r(IS_(k-2)) of that step (written by the previous start, permuted and
// wrapped with the atoms by every list rebuild), so u is a plain difference.
// From the second fine step of a call on; before that there is no history
// and u = 0 (k_lctl then rejects the start).  Same tail as the network:
// dl, partials, snapshot, plain start.  Slots of the linear-response start
// take u = 0 here: the plain start only (the solve follows, linear.hip).
template <int D>
__global__ __launch_bounds__(kBlock) void k_lextrap(LearnArgs a) {
  const int2 bt = a.blocks[blockIdx.x];
  if (bt.x < 0) return;
  const State* st = a.state + bt.x;
  if (st->phase != PH_LDESC) return;
  const Geom g = a.geom[bt.x];
  __shared__ double red[kLearnParts][4];
  const int li = bt.y * kBlock + threadIdx.x;
  const bool live = li < g.n;
  double ux = 0.0, uy = 0.0, uz = 0.0;
  if (live && st->start_mode == kStartExtrap && st->step >= 2) {
    const int64_t gi = g.atom_off + li;
    const double4 p = a.pos4[gi], q = a.alt4[gi];
    ux = (p.x - q.x) / g.dgamma;
    uy = (p.y - q.y) / g.dgamma;
    if (D == 3) uz = (p.z - q.z) / g.dgamma;
  }
  predicted_start<D>(a, st, g, bt, li, live, ux, uy, uz, red);
}

// Per slot of the selection in PH_LDESC: mean u_hat over the slot (block
// partials in block order), the pre-checks of the learned (or extrapolated)
// start, strain index k + 1 (the plain start is in place), phase PH_LPLAIN.
__global__ __launch_bounds__(kBlock) void k_lctl(LearnArgs a) {
  const int rep = a.sel[blockIdx.x];
  State* st = a.state + rep;
  if (st->phase != PH_LDESC) return;
  const Geom g = a.geom[rep];
  double v[kLearnParts] = {0, 0, 0, 0, 0, 0};
  // each thread sums a contiguous run of blocks, runs combined in thread order
  const int per = (g.nblocks + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * per, b1 = min(g.nblocks, b0 + per);
  for (int b = b0; b < b1; ++b) {
    const double* s = a.lpart + (int64_t)(g.block0 + b) * kLearnParts;
    v[0] += s[0];
    v[1] += s[1];
    v[2] += s[2];
    v[3] = fmax(v[3], s[3]);
    v[4] = fmax(v[4], s[4]);
    v[5] = fmax(v[5], s[5]);
  }
  // fixed-order combine of the per-thread runs: thread 0 walks them in LDS
  __shared__ double runs[kBlock][kLearnParts];
  for (int k = 0; k < kLearnParts; ++k) runs[threadIdx.x][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[kLearnParts] = {0, 0, 0, 0, 0, 0};
    for (int t = 0; t < kBlock; ++t) {
      s[0] += runs[t][0];
      s[1] += runs[t][1];
      s[2] += runs[t][2];
      s[3] = fmax(s[3], runs[t][3]);
      s[4] = fmax(s[4], runs[t][4]);
      s[5] = fmax(s[5], runs[t][5]);
    }
    st->lmean[0] = s[0] / (double)g.n;
    st->lmean[1] = s[1] / (double)g.n;
    st->lmean[2] = s[2] / (double)g.n;
    // the extrapolated start needs the previous step's displacement
    const bool hist = st->start_mode != kStartExtrap || st->step >= 2;
    const bool ok = hist && s[4] == 0.0 && isfinite(s[0] + s[1] + s[2]) &&
                    sqrt(s[3]) * g.dgamma <= a.max_move;
    st->learn_ok = ok ? 1 : 0;
    st->k += 1;
    st->phase = PH_LPLAIN;
  }
}

// ---------------------------------------------------------------------------
// Non-affine targets, one thread per atom id.
template <int D>
__global__ __launch_bounds__(kBlock) void k_ltargets(const Geom* geom, int ra, int rb, int n,
                                                     const double4* pos4, const int32_t* inv,
                                                     AffineMap f, Box bx, float* out) {
  const int aid = blockIdx.x * kBlock + threadIdx.x;
  if (aid >= n) return;
  const Geom ga = geom[ra], gb = geom[rb];
  const double4 pa = pos4[ga.atom_off + inv[ga.atom_off + aid]];
  const double4 pb = pos4[gb.atom_off + inv[gb.atom_off + aid]];
  double xa, ya;
  if (f.m10 == 0.0 && f.m00 == 1.0 && f.m11 == 1.0) {
    xa = pa.x + f.m01 * pa.y;
    ya = pa.y;
  } else {
    xa = f.m00 * pa.x + f.m01 * pa.y;
    ya = f.m10 * pa.x + f.m11 * pa.y;
  }
  double dx = pb.x - xa, dy = pb.y - ya, dz = (D == 3) ? pb.z - pa.z : 0.0;
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
  const double shear = f.scale;
  float* o = out + (int64_t)aid * D;
  o[0] = (float)(dx / shear);
  o[1] = (float)(dy / shear);
  if (D == 3) o[2] = (float)(dz / shear);
}

// ---------------------------------------------------------------------------
// Training.

// Column sums of x ([n][ld], columns c < C) over row chunks, FP64, over the
// rows with keep[r] = 1 (all rows if keep is null); pass 1 (mean given)
// sums (x - mean)^2.  part[blk * 64 + c]; the chunk's row count at
// part[kStatBlocks * 64 + blk].
constexpr int kStatBlocks = 256;

__global__ __launch_bounds__(kBlock) void k_colsum(const float* x, int64_t n, int C, int ld,
                                                   const double* mean, const uint8_t* keep,
                                                   double* part) {
  const int tid = threadIdx.x;
  const int cols = (C > 4) ? 64 : 4;
  const int col = tid % cols, rg = tid / cols, ngr = kBlock / cols;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  double s = 0.0, cnt = 0.0;
  if (col < C) {
    const double mu = mean ? mean[col] : 0.0;
    for (int64_t r = r0 + rg; r < r1; r += ngr) {
      if (keep && !keep[r]) continue;
      const double v = (double)x[r * ld + col];
      s += mean ? (v - mu) * (v - mu) : v;
      cnt += 1.0;
    }
  }
  __shared__ double sh[kBlock], shc[kBlock];
  sh[tid] = s;
  shc[tid] = cnt;
  __syncthreads();
  if (tid < cols && tid < C) {
    double t = 0.0, tc = 0.0;
    for (int g = 0; g < ngr; ++g) {
      t += sh[g * cols + tid];
      tc += shc[g * cols + tid];
    }
    part[(int64_t)blockIdx.x * 64 + tid] = t;
    if (tid == 0) part[(int64_t)kStatBlocks * 64 + blockIdx.x] = tc;
  }
}

// Combine the chunk sums in chunk order: pass 0 -> FP64 mean; pass 1 ->
// FP64 std (population) and the FP32 mean and std of the network (std 1
// where the spread is zero).
__global__ void k_colfin(const double* part, int nblk, int C, int pass, double* mean64,
                         double* std64, float* fmean, float* fstd) {
  const int c = threadIdx.x;
  if (c >= C) return;
  double s = 0.0, cnt = 0.0;
  for (int b = 0; b < nblk; ++b) {
    s += part[(int64_t)b * 64 + c];
    cnt += part[(int64_t)kStatBlocks * 64 + b];
  }
  if (pass == 0) {
    mean64[c] = s / cnt;
  } else {
    const double sd = sqrt(s / cnt);
    std64[c] = sd;
    fmean[c] = (float)mean64[c];
    fstd[c] = (float)(sd > 0.0 ? sd : 1.0);
  }
}

// keep[r] = 1 if every component of sample r lies within kappa std of the mean.
__global__ __launch_bounds__(kBlock) void k_trim(const float* t, int64_t n, int C,
                                                 const double* mean64, const double* std64,
                                                 double kappa, uint8_t* keep) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  bool in = true;
  for (int c = 0; c < C; ++c)
    in = in && fabs((double)t[r * C + c] - mean64[c]) <= kappa * std64[c];
  keep[r] = in ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_tprep(TrainArgs a) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= a.n) return;
  const MlpDev* M = a.mlp;
  const float* x = a.feat + r * kFeat;
  uint16_t* z = a.z + r * kFeat;
  for (int f = 0; f < kFeat; ++f) z[f] = f2bf((x[f] - M->fmean[f]) / M->fstd[f]);
  for (int c = 0; c < 4; ++c)
    a.t[r * 4 + c] = (c < a.dim) ? (a.tgt[r * a.dim + c] - M->tmean[c]) / M->tstd[c] : 0.0f;
}

constexpr int kS64 = 64 + 8;    // stride of [feature][row] buffers (64 rows)
constexpr int kGS = 32 + 8;     // stride of the output-error rows

// Forward and backward of 64 samples (4 wavefronts x 16 rows), then this
// block's share of every gradient: dW = X^T dY over its 64 rows on the
// matrix cores, bias gradients as FP64 sums; written to part[blockIdx.x].
__global__ __launch_bounds__(kBlock) void k_tfb(TrainArgs a) {
  const MlpDev* M = a.mlp;
  __shared__ __attribute__((aligned(16))) uint16_t zT[kFeat][kS64];
  __shared__ __attribute__((aligned(16))) uint16_t h1r[64][kHS];
  __shared__ __attribute__((aligned(16))) uint16_t h1T[kHid][kS64];
  __shared__ __attribute__((aligned(16))) uint16_t h2r[64][kHS];  // later dL/da2 rows
  __shared__ __attribute__((aligned(16))) uint16_t h2T[kHid][kS64];
  __shared__ __attribute__((aligned(16))) uint16_t gr[64][kGS];
  __shared__ __attribute__((aligned(16))) uint16_t gT[16][kS64];
  __shared__ __attribute__((aligned(16))) uint16_t d2T[kHid][kS64];
  __shared__ __attribute__((aligned(16))) uint16_t d1T[kHid][kS64];
  __shared__ double bsum[4][2 * kHid + 4];
  __shared__ double lsum[4];
  const int tid = threadIdx.x, w = tid / 64, l = tid % 64;
  const int lr = l & 15, lg = l >> 4, lk = 8 * lg;
  const int rw = w * 16;                              // first row of this wave
  const int rowA = blockIdx.x * 64 + rw + lr;         // batch row of this lane's A fragment
  const bool liveA = rowA < a.rows;
  const int64_t sA = liveA ? (int64_t)a.order[a.b0 + rowA] : 0;
  // ---- layer 1 (A from global z; also the transposed copy zT)
  bf16x8 z0, z1;
  {
    uint4 q0 = make_uint4(0, 0, 0, 0), q1 = q0;
    if (liveA) {
      q0 = *reinterpret_cast<const uint4*>(a.z + sA * kFeat + lk);
      q1 = *reinterpret_cast<const uint4*>(a.z + sA * kFeat + lk + 32);
    }
    const uint32_t qa[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      zT[lk + 2 * j][rw + lr] = (uint16_t)(qa[j] & 0xffffu);
      zT[lk + 2 * j + 1][rw + lr] = (uint16_t)(qa[j] >> 16);
      zT[32 + lk + 2 * j][rw + lr] = (uint16_t)(qa[4 + j] & 0xffffu);
      zT[32 + lk + 2 * j + 1][rw + lr] = (uint16_t)(qa[4 + j] >> 16);
    }
    z0 = *reinterpret_cast<const bf16x8*>(&q0);
    z1 = *reinterpret_cast<const bf16x8*>(&q1);
  }
  f32x4 a1[8], a2[8];
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    const uint16_t* wb = M->w1t + (nt * 16 + lr) * kFeat + lk;
    f32x4 acc = mma(z0, ld8(wb), zero4());
    acc = mma(z1, ld8(wb + 32), acc);
    const int col = nt * 16 + lr;
    const float b = M->b1[col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a1[nt][i] = acc[i] + b;
      const uint16_t h = f2bf(silu(a1[nt][i]));
      h1r[rw + 4 * lg + i][col] = h;
      h1T[col][rw + 4 * lg + i] = h;
    }
  }
  __syncthreads();
  // ---- layer 2
  bf16x8 hA[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) hA[kk] = ld8(&h1r[rw + lr][kk * 32 + lk]);
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    f32x4 acc = zero4();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      acc = mma(hA[kk], ld8(M->w2t + (nt * 16 + lr) * kHid + kk * 32 + lk), acc);
    const int col = nt * 16 + lr;
    const float b = M->b2[col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a2[nt][i] = acc[i] + b;
      const uint16_t h = f2bf(silu(a2[nt][i]));
      h2r[rw + 4 * lg + i][col] = h;
      h2T[col][rw + 4 * lg + i] = h;
    }
  }
  __syncthreads();
  // ---- layer 3 and the output error g = clip(y - t) / (rows d)
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) hA[kk] = ld8(&h2r[rw + lr][kk * 32 + lk]);
  f32x4 y = zero4();
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) y = mma(hA[kk], ld8(M->w3t + lr * kHid + kk * 32 + lk), y);
  const int c = lr;
  const float bd = (float)(a.rows * a.dim);
  double gsum = 0.0, lossw = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = blockIdx.x * 64 + rw + 4 * lg + i;
    float gv = 0.0f;
    if (c < a.dim && row < a.rows && (!a.keep || a.keep[a.order[a.b0 + row]])) {
      const int64_t s = a.order[a.b0 + row];
      const float e = (y[i] + M->b3[c]) - a.t[s * 4 + c];
      const float ae = fabsf(e);
      lossw += (ae <= a.delta) ? 0.5 * (double)e * (double)e
                               : (double)a.delta * ((double)ae - 0.5 * (double)a.delta);
      gv = fminf(fmaxf(e, -a.delta), a.delta) / bd;
    }
    gsum += (double)gv;
    const uint16_t gb = f2bf(gv);
    gr[rw + 4 * lg + i][c] = gb;
    gr[rw + 4 * lg + i][16 + c] = 0;
    gT[c][rw + 4 * lg + i] = gb;
  }
  // bias gradient of layer 3 (columns c) and the loss: fixed-order sums
  gsum += __shfl_xor(gsum, 16, 64);
  gsum += __shfl_xor(gsum, 32, 64);
  for (int o = 32; o > 0; o >>= 1) lossw += __shfl_xor(lossw, o, 64);
  if (l < 4) bsum[w][2 * kHid + l] = gsum;
  if (l == 0) lsum[w] = lossw;
  __syncthreads();
  // ---- dL/dh2 = g W3^T, dL/da2 = dL/dh2 silu'(a2)
  {
    const bf16x8 gA = ld8(&gr[rw + lr][lk]);
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
      const f32x4 dh = mma(gA, ld8(M->w3n + (nt * 16 + lr) * 32 + lk), zero4());
      const int col = nt * 16 + lr;
      double bs = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float dz = dh[i] * dsilu(a2[nt][i]);
        bs += (double)dz;
        const uint16_t hb = f2bf(dz);
        h2r[rw + 4 * lg + i][col] = hb;
        d2T[col][rw + 4 * lg + i] = hb;
      }
      bs += __shfl_xor(bs, 16, 64);
      bs += __shfl_xor(bs, 32, 64);
      if (l < 16) bsum[w][kHid + col] = bs;
    }
  }
  __syncthreads();
  // ---- dL/dh1 = dL/da2 W2^T, dL/da1 = dL/dh1 silu'(a1)
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) hA[kk] = ld8(&h2r[rw + lr][kk * 32 + lk]);
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    f32x4 dh = zero4();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      dh = mma(hA[kk], ld8(M->w2n + (nt * 16 + lr) * kHid + kk * 32 + lk), dh);
    const int col = nt * 16 + lr;
    double bs = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float dz = dh[i] * dsilu(a1[nt][i]);
      bs += (double)dz;
      d1T[col][rw + 4 * lg + i] = f2bf(dz);
    }
    bs += __shfl_xor(bs, 16, 64);
    bs += __shfl_xor(bs, 32, 64);
    if (l < 16) bsum[w][col] = bs;
  }
  __syncthreads();
  // ---- weight gradients over the block's 64 rows (K = 64: two steps)
  float* P = a.part + (int64_t)blockIdx.x * (kNumParams + 1);
  // 104 output tiles: dW3 (8: 128 x 16), dW2 (64: 128 x 128), dW1 (32: 64 x 128)
  for (int tt = w; tt < 104; tt += 4) {
    const uint16_t *A, *B;
    int m0, n0, off, ldo, nmax;
    if (tt < 8) {
      m0 = tt * 16; n0 = 0;
      A = &h2T[m0 + lr][0]; B = &gT[lr][0];
      off = kOffW3; ldo = 3; nmax = 3;
    } else if (tt < 72) {
      const int q = tt - 8;
      m0 = (q / 8) * 16; n0 = (q % 8) * 16;
      A = &h1T[m0 + lr][0]; B = &d2T[n0 + lr][0];
      off = kOffW2; ldo = kHid; nmax = kHid;
    } else {
      const int q = tt - 72;
      m0 = (q / 8) * 16; n0 = (q % 8) * 16;
      A = &zT[m0 + lr][0]; B = &d1T[n0 + lr][0];
      off = kOffW1; ldo = kHid; nmax = kHid;
    }
    f32x4 acc = mma(ld8(A + lk), ld8(B + lk), zero4());
    acc = mma(ld8(A + 32 + lk), ld8(B + 32 + lk), acc);
    const int n = n0 + lr;
    if (n < nmax) {
#pragma unroll
      for (int i = 0; i < 4; ++i) P[off + (m0 + 4 * lg + i) * ldo + n] = acc[i];
    }
  }
  // bias gradients and loss, waves combined in order
  if (tid < kHid) {
    P[kOffB1 + tid] = (float)(bsum[0][tid] + bsum[1][tid] + bsum[2][tid] + bsum[3][tid]);
    P[kOffB2 + tid] = (float)(bsum[0][kHid + tid] + bsum[1][kHid + tid] + bsum[2][kHid + tid] +
                              bsum[3][kHid + tid]);
  }
  if (tid < 3)
    P[kOffB3 + tid] = (tid < a.dim) ? (float)(bsum[0][2 * kHid + tid] + bsum[1][2 * kHid + tid] +
                                             bsum[2][2 * kHid + tid] + bsum[3][2 * kHid + tid])
                                    : 0.0f;
  if (tid == 0) P[kNumParams] = (float)(lsum[0] + lsum[1] + lsum[2] + lsum[3]);
}

// The BF16 copies and FP32 biases of parameter p from its master value.
__device__ __forceinline__ void sync_param(int p, float wv, MlpDev* M) {
  const uint16_t h = f2bf(wv);
  if (p < kOffB1) {
    const int i = p / kHid, o = p % kHid;
    M->w1t[o * kFeat + i] = h;
  } else if (p < kOffW2) {
    M->b1[p - kOffB1] = wv;
  } else if (p < kOffB2) {
    const int q = p - kOffW2, i = q / kHid, o = q % kHid;
    M->w2t[o * kHid + i] = h;
    M->w2n[i * kHid + o] = h;
  } else if (p < kOffW3) {
    M->b2[p - kOffB2] = wv;
  } else if (p < kOffB3) {
    const int q = p - kOffW3, i = q / 3, o = q % 3;
    const bool live = o < M->dim;
    M->w3t[o * kHid + i] = live ? h : (uint16_t)0;
    M->w3n[i * 32 + o] = live ? h : (uint16_t)0;
  } else {
    const int o = p - kOffB3;
    M->b3[o] = (o < M->dim) ? wv : 0.0f;
  }
}

// Gradient = partials summed in block order; then Adam (FP32, the order of
// operations of Kingma and Ba's Algorithm 1) and the BF16 copies.  With
// grad_out set, only the gradient is written.
__global__ __launch_bounds__(kBlock) void k_tadam(TrainArgs a) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p == 0 && a.loss_acc) {
    double s = 0.0;
    for (int b = 0; b < a.nblk; ++b) s += (double)a.part[(int64_t)b * (kNumParams + 1) + kNumParams];
    *a.loss_acc += s / ((double)a.rows * (double)a.dim);
  }
  if (p >= kNumParams) return;
  float g = 0.0f;
  for (int b = 0; b < a.nblk; ++b) g += a.part[(int64_t)b * (kNumParams + 1) + p];
  if (a.grad_out) {
    a.grad_out[p] = g;
    return;
  }
  const float m = a.beta1 * a.m[p] + (1.0f - a.beta1) * g;
  const float gg = (1.0f - a.beta2) * g;
  const float v = a.beta2 * a.v[p] + gg * g;
  const float mh = m / a.c1;
  const float vh = v / a.c2;
  const float step = (a.lr * mh) / (sqrtf(vh) + a.eps);
  const float wv = a.master[p] - step;
  a.m[p] = m;
  a.v[p] = v;
  a.master[p] = wv;
  sync_param(p, wv, a.mlp);
}

// All BF16 copies and biases from the masters; the padding that no
// parameter maps to (output columns 3..15) is cleared.
__global__ __launch_bounds__(kBlock) void k_mlp_sync(const float* master, MlpDev* M) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= 3 * kHid && p < kOutPad * kHid) M->w3t[p] = 0;
  if (p < kHid * 32 && (p % 32) >= 3) M->w3n[p] = 0;
  if (p >= 3 && p < kOutPad) M->b3[p] = 0.0f;
  if (p < kNumParams) sync_param(p, master[p], M);
}

__global__ __launch_bounds__(kBlock) void k_zero_words(uint32_t* p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = 0u;
}

}  // namespace

void launch_zero_words(uint32_t* p, int64_t words, hipStream_t s) {
  if (words <= 0) return;
  const int64_t nb = std::min<int64_t>((words + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)nb), dim3(kBlock), 0, s, p, words);
}

void launch_ldesc(const LearnArgs& a, int32_t ntiles, int32_t dim, hipStream_t s) {
  if (ntiles <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_ldesc<3>, dim3(ntiles), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_ldesc<2>, dim3(ntiles), dim3(kBlock), 0, s, a);
}

void launch_lmlp(const LearnArgs& a, int32_t nblk, int32_t dim, hipStream_t s) {
  if (nblk <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_lmlp<3>, dim3(nblk), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_lmlp<2>, dim3(nblk), dim3(kBlock), 0, s, a);
}

void launch_lextrap(const LearnArgs& a, int32_t nblk, int32_t dim, hipStream_t s) {
  if (nblk <= 0) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_lextrap<3>, dim3(nblk), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_lextrap<2>, dim3(nblk), dim3(kBlock), 0, s, a);
}

void launch_lctl(const LearnArgs& a, hipStream_t s) {
  if (a.nsel <= 0) return;
  hipLaunchKernelGGL(k_lctl, dim3(a.nsel), dim3(kBlock), 0, s, a);
}

void launch_ltargets(const Geom* geom, int32_t ra, int32_t rb, int32_t n, const double4* pos4,
                     const int32_t* inv, int32_t dim, const AffineMap& f, const Box& box, float* out,
                     hipStream_t s) {
  const int nb = (n + kBlock - 1) / kBlock;
  if (dim == 3)
    hipLaunchKernelGGL(k_ltargets<3>, dim3(nb), dim3(kBlock), 0, s, geom, ra, rb, n, pos4, inv, f,
                       box, out);
  else
    hipLaunchKernelGGL(k_ltargets<2>, dim3(nb), dim3(kBlock), 0, s, geom, ra, rb, n, pos4, inv, f,
                       box, out);
}

void launch_train_stats(const TrainArgs& a, hipStream_t s) {
  double* mean64 = a.stats;
  double* std64 = a.stats + 68;
  const int nb = (int)std::min<int64_t>(kStatBlocks, std::max<int64_t>(1, (a.n + 255) / 256));
  auto stats = [&](const float* x, int C, int off, const uint8_t* keep, float* fm, float* fs) {
    hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(kBlock), 0, s, x, a.n, C, C, (const double*)nullptr,
                       keep, a.stat_part);
    hipLaunchKernelGGL(k_colfin, dim3(1), dim3(64), 0, s, a.stat_part, nb, C, 0, mean64 + off,
                       std64 + off, fm, fs);
    hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(kBlock), 0, s, x, a.n, C, C,
                       (const double*)(mean64 + off), keep, a.stat_part);
    hipLaunchKernelGGL(k_colfin, dim3(1), dim3(64), 0, s, a.stat_part, nb, C, 1, mean64 + off,
                       std64 + off, fm, fs);
  };
  stats(a.feat, kFeat, 0, nullptr, a.mlp->fmean, a.mlp->fstd);
  // targets: trimmed statistics; the final window decides which samples train
  stats(a.tgt, a.dim, 64, nullptr, a.mlp->tmean, a.mlp->tstd);
  const unsigned tb = (unsigned)((a.n + kBlock - 1) / kBlock);
  for (int r = 0; r < kTrimRounds; ++r) {
    hipLaunchKernelGGL(k_trim, dim3(tb), dim3(kBlock), 0, s, a.tgt, a.n, a.dim,
                       (const double*)(mean64 + 64), (const double*)(std64 + 64), kTrimKappa, a.keep);
    stats(a.tgt, a.dim, 64, a.keep, a.mlp->tmean, a.mlp->tstd);
  }
  hipLaunchKernelGGL(k_trim, dim3(tb), dim3(kBlock), 0, s, a.tgt, a.n, a.dim,
                     (const double*)(mean64 + 64), (const double*)(std64 + 64), kTrimKappa, a.keep);
}

void launch_train_prep(const TrainArgs& a, hipStream_t s) {
  const int64_t nb = (a.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_tprep, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
}

void launch_train_batch(const TrainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_tfb, dim3(a.nblk), dim3(kBlock), 0, s, a);
}

void launch_train_update(const TrainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_tadam, dim3((kNumParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}

void launch_mlp_sync(const float* master, MlpDev* mlp, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_sync, dim3((kNumParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     master, mlp);
}

}  // namespace aqs
