// kernels.h -- host-side launchers of the HIP kernels (internal).
#pragma once

#include "engine.h"
#include "tiles.h"

namespace aqs {

// Rebuild of cell lists and neighbour lists for a set of slots.
constexpr int kGridInts = 6;  // per slot: nc0, nc1, nc2, tiles per row, tiles, list mode

struct RebuildArgs {
  const int2* blocks;   // launch table over the atoms of the slots to rebuild
  int32_t nblk;         // entries of the launch table
  const int2* tiles;    // launch table over the force tiles of those slots
  int32_t ntile_blk;
  const int32_t* reps;  // slots to rebuild
  int32_t nreps;
  const Geom* geom;
  State* state;
  double4* pos4;
  double4* xref4;       // positions at the build (list validity test)
  double* vx; double* vy; double* vz;
  int32_t* id; int32_t* inv;
  int32_t* nbc;
  uint32_t* nbl;
  uint2* nbp;           // packed lists (engine.h)
  TileHdr* thdr;        // per force tile (tile_off + t)
  uint32_t* hidx;       // compact halo per force tile (kHaloCap slots): j | code << 24
  int32_t* tord;        // per atom: the tile's atoms by decreasing list length
  int32_t* cell_count;  // per cell (cell_off + c)
  int32_t* cell_start;  // per cell + 1 per slot (cell_off + slot_index + c)
  int32_t* cell_of;     // per atom
  int32_t* order;       // per atom
  double4* tpos4;       // per atom scratch
  double* tvx; double* tvy; double* tvz;
  int32_t* tid_;
  double* upart;
  int32_t* overflow;
  PairParams pp[4];
  double skin;
  int32_t max_nb;
  int32_t dim;
  int32_t resume;       // 1: slots in PH_REBUILD go back to the phase they left
  // learned-start per-atom buffers permuted with the atoms (may be null):
  // predicted displacement, and the saved plain start (also wrapped with
  // the positions, so a revert restores the wrapped plain start bit for bit)
  double* dlx; double* dly; double* dlz;
  double* tdlx; double* tdly; double* tdlz;
  double4* alt4; double4* talt4;
};

void launch_rebuild(const RebuildArgs& a, int32_t max_cells_per_slot, hipStream_t s,
                    const int32_t* nc3_dev);

// One FIRE iteration: force + control over the force tiles (a.ftiles), then
// the update over the 256-atom blocks (a.blocks).
// with events e0, e1: the kernel's own start and end (hipExtLaunchKernelGGL)
void launch_force(const IterArgs& a, int32_t ntiles, int32_t dim, hipStream_t s,
                  hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// per-slot reduction of the force partials and the control, state updated in
// place (after launch_force; the single evaluation of aqs_energy_forces)
void launch_control(const IterArgs& a, hipStream_t s);
// one iteration's control and move over the update table (after launch_force):
// reads a.state / a.cgst / a.upart, writes a.state_out / a.cgst_out / a.upart_out
void launch_step(const IterArgs& a, int32_t nblk, int32_t dim, hipStream_t s,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// dynamic LDS bytes per force block that leave at most `blocks` force blocks
// per CU plus room for one more (0 if none can)
int32_t force_lds_pad(int32_t dim, int32_t tpa, int32_t blocks);

// Affine shear x += dg_r y of whole slots (host-driven level I step).
void launch_affine(const int2* blocks, int32_t nblk, const Geom* geom, double4* pos4,
                   const double* dg_per_slot, hipStream_t s);

// v = 0 and partials of the update = 0 for the slots of the launch table.
void launch_reset_iter(const int2* blocks, int32_t nblk, const Geom* geom, double* vx,
                       double* vy, double* vz, double* upart, int32_t dim, hipStream_t s);

// Copy slot src into slot dst (same n), including order and inverse.
void launch_copy_slot(const Geom* geom, int32_t src, int32_t dst, int32_t n, double4* pos4,
                      int32_t* id, int32_t* inv, hipStream_t s);

// Max minimum-image distance per block between two slots (atom-id order).
void launch_compare(const Geom* geom, int32_t ra, int32_t rb, int32_t n, const double4* pos4,
                    const int32_t* inv, const Box& box, int32_t dim, double* part, hipStream_t s);

// Energy and full virial per block of one slot: 1 + 9 doubles per block.
void launch_virial(const IterArgs& a, int32_t rep, int32_t nblocks, int32_t dim, const Box& box,
                   double* part, hipStream_t s);

}  // namespace aqs
