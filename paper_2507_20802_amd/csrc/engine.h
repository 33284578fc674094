// engine.h -- device-side data layout shared by the HIP kernels and the host
// side of the AQS engine (not part of the public ABI; see include/aqs.h).
//
// Layout in HBM (one context = one batch of slots):
//   per-atom arrays, every slot padded to a multiple of kBlock atoms:
//     pos4   double4 (x, y, z, type)  AoS, the gather target of the force loop
//     vx,vy,vz, fx,fy,fz              SoA FP64, streamed coalesced
//     id     int32, atom id held by each sorted position ("slot order")
//     inv    int32, sorted position of each atom id
//     nbc    int32, neighbour counts per atom (A | B << 16)
//   neighbour lists per slot, the nA neighbours of type A first and the nB
//     of type B second, nbc = nA | nB << 16 (the neighbour's type is that of
//     its segment):
//   - packed list (force tiles with an LDS halo): max_nb / 4 group rows x
//     npad columns of 8 bytes, four 16-bit entries each, column-major (group
//     row g of column c at g*npad + c) so a wavefront reads 512 consecutive
//     bytes; entry = 8 x halo slot, the byte offset of the slot in the halo
//     coordinate arrays; A neighbours fill group rows 0.. upward, B
//     neighbours group rows max_nb/4 - 1 downward, the last group of each
//     padded with the far fill slot; column c belongs to atom tord[c] (each
//     tile's atoms ordered by decreasing list length; nbc is indexed by
//     column too);
//   - word list: max_nb x npad uint32, row k of column c at k*npad + c; A
//     neighbours in rows 0.. upward, B neighbours rows max_nb - 1 downward;
//     entry = j | (image code << 24) (tiles without an LDS halo, whose
//     columns are the atoms in tile order), or, for tiles with a halo, the
//     builder's candidate numbers (scratch)
//   xref4  double4, positions at the last list build (validity test)
//   per-block partial sums, per-slot counters, per-slot state and geometry.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aqs {

constexpr int kBlock = 256;           // atoms per workgroup (4 wavefronts)
constexpr int kWave = 64;
constexpr int kForceParts = 8;        // doubles per tile partial of the force kernel
constexpr int kMaxTPA = 8;            // threads per atom of the force kernel: 1, 2, 4 or 8
// LDS halo capacity (atoms) of a force tile: its compact halo (the atoms
// some list of the tile names) plus the far fill slot
constexpr int kHaloCap3 = 1248;       // 3D (with the rest of the force kernel's LDS: 5 blocks per CU)
constexpr int kHaloCap2 = 1024;       // 2D
__host__ __device__ constexpr int halo_cap(int dim) { return dim == 3 ? kHaloCap3 : kHaloCap2; }
constexpr uint32_t kIdxMask = 0x00FFFFFFu;
constexpr int kCodeShift = 24;
constexpr int kGroup = 4;             // entries per 8-byte group of the packed list
constexpr int kListAlign = 32;        // max_nb is a multiple of kGroup x kMaxTPA
// Blocks of one launch are dealt to the XCDs (dies, each with its own L2)
// round robin: hardware block b runs on XCD b mod kXcds.
constexpr int kXcds = 8;

// Item of hardware block b in a launch over the n items of one slot, placed
// like the launch tables over all XCDs: each XCD takes a contiguous run of
// ceil(n / kXcds) items.  -1: no item (the block exits).
__host__ __device__ inline int one_slot_item(int b, int n) {
  const int per = (n + kXcds - 1) / kXcds;
  const int t = (b % kXcds) * per + b / kXcds;
  return t < n ? t : -1;
}

// phases of a slot's device state machine
enum Phase : int32_t {
  PH_IDLE = 0,      // not part of the running call
  PH_FIRE = 1,      // evaluate forces; control; FIRE update
  PH_ADVANCE = 2,   // update applies the fine affine step (and snapshot)
  PH_FINISH = 3,    // update takes the snapshot only; next force kernel -> DONE
  PH_STOP = 4,      // update applies the last FIRE step; next force kernel -> DONE
  PH_DONE = 5,
  PH_REBUILD = 6,   // neighbour list no longer valid; waits for the host
  PH_EVAL = 7,      // one force evaluation without FIRE control
  PH_ENERGY = 11,   // evaluate again with the energy, then record the pending outcome
  PH_LDESC = 8,     // learned start: descriptors + network pending at the IS
  PH_LMOVE = 9,     // learned start: update moved plain start -> learned start;
                    // evaluate there, then accept (FIRE) or revert
  PH_LREVERT = 10,  // learned start rejected: update restores the plain start
  PH_LPLAIN = 12,   // learned start: evaluate at the plain start (reference E, max |F|)
  PH_CG = 13,       // evaluate forces; conjugate-gradient control; CG update
  PH_LPROBE = 14,   // linear-response start: forces at a probe of the Hessian
                    // solve (the host drives the solve; no control)
};

// minimiser of a slot (State::minimizer; AQS_MIN_* of the public header)
constexpr int32_t kMinFire = 0, kMinCG = 1;

// start of a minimisation (StepRecord::start; State::start_mode): the affine
// image, the learned start, the affine image after a learned or extrapolated
// start was rejected, the extrapolated start
constexpr int32_t kStartPlain = 0, kStartLearned = 1, kStartFallback = 2, kStartExtrap = 3,
                  kStartLinear = 4;

// a start predicted at each inherent structure before the next fine step
__host__ __device__ inline bool predicted_start_mode(int32_t m) {
  return m == kStartLearned || m == kStartExtrap || m == kStartLinear;
}

__host__ __device__ inline bool phase_energy(int32_t ph) {  // evaluation also sums E
  return ph == PH_EVAL || ph == PH_ENERGY || ph == PH_LPLAIN || ph == PH_LMOVE;
}
__host__ __device__ inline bool phase_force(int32_t ph) {   // the force kernel evaluates
  return phase_energy(ph) || ph == PH_FIRE || ph == PH_CG || ph == PH_ADVANCE ||
         ph == PH_LREVERT || ph == PH_LPROBE;
}

// Scalars of a slot's linear-response solve (conjugate gradients on
// H u = f(x0), Eqs. 7-8): written by the owner block of its kernels, read by
// every block of the next.
struct LinState {
  double rr[2];   // |r|^2 of the current residual, by parity of the iteration
  double bb;      // |f(x0)|^2
  int32_t iters;  // completed updates of u
  int32_t done;   // the solve has stopped (converged or non-positive curvature)
  int32_t probes; // Hessian-vector products formed (two force evaluations each)
  int32_t pad_;
};

// static per-slot geometry
struct Geom {
  int64_t atom_off;   // first atom in the per-atom arrays (multiple of kBlock)
  int64_t nb_off;     // first entry of the neighbour list
  int32_t n;          // atoms
  int32_t npad;       // n rounded up to kBlock
  int32_t block0;     // first block index (partials are per global block)
  int32_t nblocks;    // npad / kBlock
  int32_t cell_off;   // first cell of this slot in the cell arrays
  int32_t cell_cap;   // cells reserved
  int32_t tile_off;   // first force tile of this slot in the tile arrays
  int32_t tile_cap;   // force tiles reserved
  double L[3];        // unstrained box edges
  double dgamma;      // fine strain increment (simple shear: x += dgamma y)
  double dgamma_y;    // 0: simple shear; else the pure shear of Eq. (17),
                      // F = [[1, dgamma], [dgamma_y, 1]] on (x, y), z unchanged
};

// dynamic per-slot state (written by the control)
struct State {
  int64_t k;          // strain index: gamma = k * dgamma
  int64_t it;         // FIRE updates in the current minimisation
  double dt, alpha;   // FIRE time step and mixing
  double cv, cf;      // pending update: v <- cv v + cf F
  double E, fmax, sxy;      // last force evaluation
  double ubound;      // sum of per-iteration max displacements since the build
  double gamma_build; // strain at the last neighbour-list build
  double E_plain, fmax_plain;  // learned start: plain-start reference values
  double lmean[3];    // learned start: mean predicted displacement per unit strain
  int32_t npos, nneg;
  int32_t restart;    // pending update backs off x -= dt v / 2, v = 0
  int32_t phase;
  int32_t status;     // outcome of the last finished minimisation
  int32_t step;       // fine step of the chain being minimised (0 = first)
  int32_t n_steps;    // fine steps to run after the first minimisation
  int32_t snap_dst;   // slot receiving the first inherent structure, or -1
  int32_t do_snap;    // pending update copies this slot into snap_dst
  int32_t nc[3];      // cell grid of the current list
  int32_t start_mode; // AQS_START_*
  int32_t start_used; // start of the minimisation in progress
  int32_t learn_ok;   // learned displacement passed its pre-checks
  int32_t pending;    // outcome recorded after the PH_ENERGY evaluation
  int32_t tiles_x;    // force tiles (row segments) per cell row
  int32_t ntiles;     // force tiles of the current grid
  int32_t list_mode;  // 0: tiles index their LDS halo; 1: global indices only
  int32_t resume_phase;  // phase to resume after a neighbour-list rebuild
  int32_t drops;      // fine steps of this call whose shear stress fell below the step before's
  double sxy_prev;    // shear stress of the last finished minimisation
  int64_t k_build;    // strain index at the last neighbour-list build
};

// Conjugate-gradient state of a slot, kept apart from State so that the FIRE
// kernels never load it.  A line search runs along d (held in v) from
// x0 = x - a d; reset at the first evaluation of every minimisation (it = 0).
struct CgState {
  double a;                 // trial step
  double alo, plo;          // last point still descending: step, phi'(step)
  double ahi, phi;          // first point past the minimum (ahi < 0: none yet)
  double p0, ff0;           // phi'(0) = -F(x0).d and |F(x0)|^2
  double aprev, p0prev;     // accepted step and phi'(0) of the previous search
  double beta, step;        // pending update: d <- F + beta d (new direction), x += step d
  int32_t dir;              // a search direction exists
  int32_t newdir;           // the pending update starts a new direction
  int32_t nls;              // evaluations in the current line search
  int32_t nfail;            // consecutive failed line searches
};

struct PairParams {   // per type pair t = 2 ti + tj
  double rc2, sig2, eps4, ucut;
};

struct FireParams {
  double dt0, dt_max, dt_min, f_inc, f_dec, alpha0, f_alpha, dmax, ftol;
  int32_t n_delay, n_neg_max, initial_delay, pad_;
  int64_t max_iter;
};

struct CgParams {
  double a_init, sigma, grow, dmax, ftol;
  int32_t ls_max, n_fail_max;
  int64_t max_iter;
};

struct StepRecord {
  int64_t iters;
  double energy, max_f, sigma_xy;
  int32_t status, start;
};

// Everything the iteration kernels need, passed by value.
struct IterArgs {
  const int2* blocks;     // update launch table: (slot, 256-atom block) or slot -1
  const int2* ftiles;     // force launch table: (slot, force tile) or slot -1
  const int32_t* sel;     // slots of the running selection (control kernel)
  int32_t nsel;
  int32_t tpa;            // threads per atom of the force kernel
  int32_t waves;          // force kernel instantiation: 4 or 5 waves per SIMD
  int32_t lds_pad;        // dynamic LDS bytes added to each force block (CU reservation)
  int32_t prio;           // 1: the critical chain of a live round (its waves issue first)
  // a lane of one slot over all XCDs: the iteration kernels compute their
  // launch-table entries (one_slot_item) instead of loading them
  int32_t one_rep;        // the slot, or -1: load the tables
  int32_t one_ntiles;     // its force tiles (current grid)
  int32_t one_nblk;       // its 256-atom blocks
  int32_t one_tile0;      // its first global tile index
  const Geom* geom;
  // State, conjugate-gradient state and displacement partials are
  // double-buffered over the iterations of a block: an iteration reads the
  // in buffers (state, cgst, upart) and writes the out buffers, and the host
  // swaps the two for the next iteration.  Home (the first buffer) is where
  // they are between blocks (blocks have an even number of iterations) and
  // where slots outside the launch keep them.
  State* state;
  State* state_out;
  State* state_home;
  double4* pos4;
  double* vx; double* vy; double* vz;
  double* fx; double* fy; double* fz;
  int32_t* id; int32_t* inv;
  const int32_t* nbc;
  const uint32_t* nbl;        // word lists (tiles without an LDS halo)
  const uint2* nbp;           // packed lists (tiles with an LDS halo); slot at nb_off / 4
  const int32_t* cell_start;  // per slot: cell_off + c, cells of the current grid
  const void* thdr;           // TileHdr per force tile (tile_off + t)
  const uint32_t* hidx;       // compact halo per force tile (kHaloCap slots): j | code << 24
  const int32_t* tord;        // list column -> atom: each tile's atoms by decreasing list length
  double* fpart;          // kForceParts per force tile (tile_off + tile)
  double* upart;          // 1 per global block (max displacement of the update)
  double* upart_out;
  unsigned long long* evals;  // atoms evaluated by force launches (statistics)
  unsigned long long* tevals; // ... by the launches timed with events (null: not timed)
  StepRecord* log;        // per slot, log_cap records
  int32_t log_cap;
  int32_t max_nb;
  PairParams pp[4];
  FireParams fire;
  CgParams cg;
  CgState* cgst;          // per slot (conjugate gradients)
  CgState* cgst_out;
  int32_t minimizer;      // kMinFire or kMinCG: every slot of the launch
  double skin, rc_max;
  // learned start (null when unused)
  double* dlx; double* dly; double* dlz;   // learned displacement per atom
  double4* alt4;                            // saved plain start
  // conjugate gradients: F at the line-search origin.  Shares the learned
  // displacement's arrays, which are dead once a minimisation runs (and are
  // permuted with the atoms by every list rebuild).
  double* gx; double* gy; double* gz;
  const double4* xref4;                     // positions at the last list build
};

__host__ __device__ inline double strain_of(int64_t k, double dgamma) {
  return (double)k * dgamma;
}

// The (x, y) block of a box H (columns are the Bravais vectors) and its z
// edge: H = [[h00, h01, 0], [h10, h11, 0], [0, 0, h22]].  Simple shear keeps
// h10 = 0; the pure shear of Eq. (17) does not.
struct Box {
  double h00, h01, h10, h11, h22;
};

// F^k for F = [[1, a], [b, 1]], k >= 0, row-major into M: square and multiply
// over the bits of k from the lowest (R <- R B when the bit is set, then
// B <- B B), each product entry X[i][0] Y[0][j] + X[i][1] Y[1][j], with no
// fused multiply-adds, so host, device and any plain FP64 evaluation in the
// same order agree bit for bit.
__host__ __device__ inline void deformation_power(double a, double b, int64_t k, double* M) {
#pragma clang fp contract(off)
  double r00 = 1.0, r01 = 0.0, r10 = 0.0, r11 = 1.0;
  double b00 = 1.0, b01 = a, b10 = b, b11 = 1.0;
  while (k > 0) {
    if (k & 1) {
      const double t00 = r00 * b00 + r01 * b10, t01 = r00 * b01 + r01 * b11;
      const double t10 = r10 * b00 + r11 * b10, t11 = r10 * b01 + r11 * b11;
      r00 = t00;
      r01 = t01;
      r10 = t10;
      r11 = t11;
    }
    const double u00 = b00 * b00 + b01 * b10, u01 = b00 * b01 + b01 * b11;
    const double u10 = b10 * b00 + b11 * b10, u11 = b10 * b01 + b11 * b11;
    b00 = u00;
    b01 = u01;
    b10 = u10;
    b11 = u11;
    k >>= 1;
  }
  M[0] = r00;
  M[1] = r01;
  M[2] = r10;
  M[3] = r11;
}

// The box of a slot at strain index k: simple shear (Eq. 16) H = [[Lx, k dgamma
// Ly], [0, Ly]] with the tilt formed in one product; pure shear (Eq. 17)
// H = F^k diag(Lx, Ly); z unchanged.
__host__ __device__ inline Box box_at(const Geom& g, int64_t k) {
#pragma clang fp contract(off)
  Box b;
  b.h22 = g.L[2];
  if (g.dgamma_y == 0.0) {
    b.h00 = g.L[0];
    b.h01 = strain_of(k, g.dgamma) * g.L[1];
    b.h10 = 0.0;
    b.h11 = g.L[1];
    return b;
  }
  double M[4];
  deformation_power(g.dgamma, g.dgamma_y, k, M);
  b.h00 = M[0] * g.L[0];
  b.h01 = M[1] * g.L[1];
  b.h10 = M[2] * g.L[0];
  b.h11 = M[3] * g.L[1];
  return b;
}

// Deformation of the (x, y) block since the list build, G = H_k H_kb^-1,
// row-major; z is not deformed.
__host__ __device__ inline void strain_since(const Geom& g, int64_t k, int64_t kb, double* G) {
#pragma clang fp contract(off)
  const Box h = box_at(g, k), b = box_at(g, kb);
  const double det = b.h00 * b.h11 - b.h01 * b.h10;
  const double i00 = b.h11 / det, i01 = -b.h01 / det, i10 = -b.h10 / det, i11 = b.h00 / det;
  G[0] = h.h00 * i00 + h.h01 * i10;
  G[1] = h.h00 * i01 + h.h01 * i11;
  G[2] = h.h10 * i00 + h.h11 * i10;
  G[3] = h.h10 * i01 + h.h11 * i11;
}

// Largest singular value of G^-1 (the most a separation can have shrunk
// under G): sigma^2 = (f + sqrt(f^2 - 4 det^2)) / 2 for the 2x2 inverse with
// squared Frobenius norm f.
__host__ __device__ inline double inverse_strain_norm(const Geom& g, int64_t k, int64_t kb) {
  double G[4];
  strain_since(g, k, kb, G);
  const double det = G[0] * G[3] - G[1] * G[2];
  const double j00 = G[3] / det, j01 = -G[1] / det, j10 = -G[2] / det, j11 = G[0] / det;
  const double f = j00 * j00 + j01 * j01 + j10 * j10 + j11 * j11;
  const double dj = j00 * j11 - j01 * j10;
  const double disc = fmax(f * f - 4.0 * dj * dj, 0.0);
  return fmax(1.0, sqrt(0.5 * (f + sqrt(disc))));
}

// An affine map of (x, y) (z unchanged) and the strain scale of the step it
// makes (the divisor of non-affine displacements per unit strain).
struct AffineMap {
  double m00, m01, m10, m11, scale;
};

// Image shift H (ix, iy, iz).
__host__ __device__ inline void box_shift(const Box& b, int ix, int iy, int iz, double* s) {
  if (b.h10 == 0.0) {
    s[0] = (double)ix * b.h00 + (double)iy * b.h01;
    s[1] = (double)iy * b.h11;
  } else {
    s[0] = (double)ix * b.h00 + (double)iy * b.h01;
    s[1] = (double)ix * b.h10 + (double)iy * b.h11;
  }
  s[2] = (double)iz * b.h22;
}

}  // namespace aqs
