// learned.h -- learned start of an AQS step (internal): descriptors, the
// per-atom network on BF16 matrix cores, its training, and the device
// phases that put the learned start between two minimisations.
//
// Network: 64 features -> 128 -> SiLU -> 128 -> SiLU -> d outputs (the
// non-affine displacement per unit strain, standardised), BF16 weights and
// layer inputs, FP32 accumulation, biases and SiLU.
#pragma once

#include <stdint.h>

#include "engine.h"

namespace aqs {

constexpr int kFeat = 64;
constexpr int kHid = 128;
constexpr int kOutPad = 16;                 // output columns of the last product
constexpr int kNumParams = kFeat * kHid + kHid + kHid * kHid + kHid + kHid * 3 + 3;
// offsets of the flat FP32 parameter vector (the order of aqs_mlp)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kFeat * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * 3;

// Device copy of the network used by the kernels.  BF16 values are stored as
// their 16 raw bits.  "t" arrays are [out][in] (k contiguous for the
// forward products), "n" arrays [in][out] (for the backward products).
struct MlpDev {
  uint16_t w1t[kHid * kFeat];       // [128 out][64 in]
  uint16_t w2t[kHid * kHid];        // [128 out][128 in]
  uint16_t w3t[kOutPad * kHid];     // [16 out][128 in], rows >= d zero
  uint16_t w2n[kHid * kHid];        // [128 in][128 out]
  uint16_t w3n[kHid * 32];          // [128 in][32 out], columns >= d zero
  float b1[kHid], b2[kHid], b3[kOutPad];
  float fmean[kFeat], fstd[kFeat];
  float tmean[4], tstd[4];
  int32_t dim, pad_[3];
};

// Arguments of the descriptor / inference kernels of the engine.
struct LearnArgs {
  const int2* blocks;       // (slot, 256-atom block) launch table
  const int2* ftiles;       // (slot, force tile) launch table
  const void* thdr;         // TileHdr per force tile
  const uint32_t* hidx;     // compact halo per force tile (kHaloCap slots): j | code << 24
  const uint32_t* nbl;      // word lists (engine.h): tiles without an LDS halo
  const uint2* nbp;         // packed lists (engine.h): tiles with an LDS halo
  const int32_t* nbc;
  const int32_t* tord;      // per tile: atoms in list order (list column -> atom)
  int32_t max_nb;
  const int32_t* sel;       // slots of the running selection
  int32_t nsel;
  int32_t mode;             // see the launchers
  const Geom* geom;
  State* state;
  double4* pos4;
  double* vx; double* vy; double* vz;
  int32_t* id; int32_t* inv;
  const int32_t* cell_start;
  const double4* xref4;
  double* upart;
  double* lpart;            // per global block: 6 doubles
  uint16_t* zbuf;           // per atom 64 BF16 features (slot order)
  double* dlx; double* dly; double* dlz;
  double4* alt4;            // saved plain start (restored on a rejected learned start)
  float* out;               // API output (atom-id order)
  const MlpDev* mlp;
  double rd2[4];            // descriptor cutoff^2 per type pair (2 ti + tj)
  double rd[4];
  double dirs[16][3];       // directions of the angular features
  double max_move;          // largest accepted |dgamma u_hat| (sigma_AA)
};

constexpr int kLearnParts = 6;
constexpr double kTrimKappa = 5.0;  // target window of the trimmed statistics, in std
constexpr int kTrimRounds = 3;   // sum u_hat (3), max |u_hat|^2, non-finite, max displacement

// Over the force-tile table (a.ftiles, ntiles entries):
// mode 0: slots in PH_LDESC, standardised BF16 features into zbuf;
// mode 1: every slot of the table, raw FP32 features into out[id * 64 + f];
// mode 2: every slot of the table, standardised BF16 features into zbuf.
void launch_ldesc(const LearnArgs& a, int32_t ntiles, int32_t dim, hipStream_t s);
// mode 0: slots in PH_LDESC: u_hat into dl, partials, snapshot, plain start;
// mode 1: every slot of the table: u_hat into out[id * d + c] (FP32).
void launch_lmlp(const LearnArgs& a, int32_t nblk, int32_t dim, hipStream_t s);
// slots in PH_LDESC: the extrapolated start (previous step's non-affine
// displacement per unit strain) into dl, partials, snapshot, plain start
void launch_lextrap(const LearnArgs& a, int32_t nblk, int32_t dim, hipStream_t s);
// per slot of the selection in PH_LDESC: mean u_hat, checks, k + 1, PH_LPLAIN
void launch_lctl(const LearnArgs& a, hipStream_t s);

// u / f.scale per atom (atom-id order, FP32 [n][dim]) from slot ra (earlier
// inherent structure) to slot rb (later one, in the box `box`),
// u = minimg(r_b - F r_a), F the affine map f of the steps between them.
void launch_ltargets(const Geom* geom, int32_t ra, int32_t rb, int32_t n, const double4* pos4,
                     const int32_t* inv, int32_t dim, const AffineMap& f, const Box& box, float* out,
                     hipStream_t s);

// ---- training -------------------------------------------------------------
struct TrainArgs {
  const float* feat;        // [n][64] raw features
  const float* tgt;         // [n][dim] raw targets
  int64_t n;
  int32_t dim;
  uint16_t* z;              // [n][64] standardised BF16 features
  float* t;                 // [n][4] standardised targets
  double* stat_part;        // [blocks][64] partial sums, then [blocks] sample counts
  double* stats;            // FP64 mean[68], std[68] (64 features then 4 target columns)
  uint8_t* keep;            // per sample: 1 = in the loss (trimmed target statistics)
  const int32_t* order;     // sample order of the epoch
  int64_t b0;               // first position of the batch in order
  int32_t rows;             // samples in the batch
  float delta;              // Huber delta
  float* part;              // [blocks][kNumParams + 1] gradient and loss partials
  int32_t nblk;             // blocks of the batch
  float* master; float* m; float* v;  // FP32 parameters and Adam moments
  MlpDev* mlp;
  float lr, beta1, beta2, eps, c1, c2;  // c = 1 - beta^t
  float* grad_out;          // gradient-only mode: the summed gradient (else null)
  double* loss_acc;         // += batch loss
};

void launch_train_stats(const TrainArgs& a, hipStream_t s);
void launch_train_prep(const TrainArgs& a, hipStream_t s);
void launch_train_batch(const TrainArgs& a, hipStream_t s);
void launch_train_update(const TrainArgs& a, hipStream_t s);
// BF16 copies and biases of the device network from the FP32 masters
void launch_mlp_sync(const float* master, MlpDev* mlp, hipStream_t s);
// words 32-bit zeros from p on (a kernel, not a memset node, so that the call
// may sit in a captured stream)
void launch_zero_words(uint32_t* p, int64_t words, hipStream_t s);

}  // namespace aqs
