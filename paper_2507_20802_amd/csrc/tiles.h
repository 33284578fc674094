// tiles.h -- force tiles and their LDS halos.
//
// A force tile is a segment of one cell row (fixed y, z): the atoms of a row
// (one contiguous range of the cell-sorted order) are cut into tiles_per_row
// segments of nearly equal atom counts (about kTileAtoms each).  Its halo is
// candidates are every (cell, periodic image) pair within one cell of the
// segment's cells [cx0, cx1]: for each of the 3^(dim-1) neighbouring rows
// (dy, dz) the cells x = cx0-1 .. cx1+1, as up to three runs -- the cells
// inside the box ("M") and, when the segment touches an x face, the wrapped
// cell on the other side ("L", image -1; "R", image +1).  Each run is a
// contiguous atom range; the runs number the candidates.
//
// The neighbour-list builder keeps, per tile, the candidates that some list
// of the tile names -- its compact halo, about half of the candidates -- and
// writes a header (TileHdr) and the compact halo as j | image code << 24.
// The force kernel stages the compact halo positions (image shift H n added)
// into LDS, and the neighbour entries of the tile's atoms hold byte offsets
// of compact halo slots.  A tile whose compact halo exceeds the LDS capacity
// (rare: dense fluctuations) keeps global indices and image codes and its
// force loop gathers from global memory.
#pragma once

#include "engine.h"

namespace aqs {

constexpr int kRuns = 27;  // (dz, dy, part): 3 x 3 x 3 (2D uses dz = 0 only)
constexpr int kTileSort = 1024;  // tiles up to this many atoms are walked by list length
constexpr int kHaloWords = 128;  // candidate bitmap of the builder: tiles with more candidates
                                 // (32 kHaloWords) keep global entries
constexpr int kRowStage = 4096;  // list words the builder stages in LDS per pass (a pass holds
                                 // whole groups: kGroup rows of up to kTileSort atoms)
constexpr int kCandCap = 32 * kHaloWords;  // candidates a tile may have and still number them
// FP32 distance test of the list builder: pairs within rc_ab + skin + this
// margin (sigma_AA) are kept, far more than the FP32 rounding of candidate
// offsets within a few cells of the tile (below 1e-5); the extra pairs lie
// beyond the cutoff and the force loop's FP64 test drops them
constexpr double kListMargin = 1e-3;

struct TileHdr {
  int32_t a0, a1;   // atom range [a0, a1) of the tile
  int32_t pad_;
  int32_t halo;     // atoms of the compact halo; -1: too large, entries are global
};

struct TileRun {
  int32_t src;      // first atom of the run (slot-local)
  int32_t count;
  int32_t off;      // candidate number of the run's first atom
  int32_t code;     // image code (ix+1) + 3 (iy+1) + 9 (iz+1)
};

// Run r = ((dz+1) * 3 + (dy+1)) * 3 + part, part 0 = L, 1 = M, 2 = R, of a
// segment with cells [cx0, cx1] in row (cy, cz).  count = 0 if absent.
template <int D>
__device__ __forceinline__ TileRun make_run(int r, int cx0, int cx1, int cy, int cz, const int* nc,
                                            const int32_t* cs) {
  TileRun run;
  run.src = 0;
  run.count = 0;
  run.off = 0;
  run.code = 13;
  const int part = r % 3, dy = (r / 3) % 3 - 1, dz = r / 9 - 1;
  if (D == 2 && dz != 0) return run;
  int ry = cy + dy, iy = 0;
  if (ry < 0) { ry += nc[1]; iy = -1; }
  else if (ry >= nc[1]) { ry -= nc[1]; iy = 1; }
  int rz = cz + dz, iz = 0;
  if (D == 3) {
    if (rz < 0) { rz += nc[2]; iz = -1; }
    else if (rz >= nc[2]) { rz -= nc[2]; iz = 1; }
  }
  const int c0 = (rz * nc[1] + ry) * nc[0];
  int xlo, xhi, ix = 0;
  if (part == 1) {
    xlo = max(0, cx0 - 1);
    xhi = min(nc[0] - 1, cx1 + 1);
  } else if (part == 0) {
    if (cx0 != 0) return run;
    xlo = xhi = nc[0] - 1;
    ix = -1;
  } else {
    if (cx1 != nc[0] - 1) return run;
    xlo = xhi = 0;
    ix = 1;
  }
  run.src = cs[c0 + xlo];
  run.count = cs[c0 + xhi + 1] - run.src;
  run.code = (ix + 1) + 3 * (iy + 1) + 9 * (iz + 1);
  return run;
}

// Run of the neighbour cell (cx + dx, row + dy, dz) of a segment cell cx.
__device__ __forceinline__ int run_of(int cx, int dx, int dy, int dz, int nc0) {
  const int x = cx + dx;
  const int part = x < 0 ? 0 : (x >= nc0 ? 2 : 1);
  return ((dz + 1) * 3 + (dy + 1)) * 3 + part;
}

// Image code c = (ix+1) + 3 (iy+1) + 9 (iz+1); shift = H (ix, iy, iz).
__device__ __forceinline__ void code_shift(int code, const Box& b, double* s) {
  const int ix = code % 3 - 1, iy = (code / 3) % 3 - 1, iz = code / 9 - 1;
  box_shift(b, ix, iy, iz, s);
}

// Stage a tile's compact halo into LDS (image shifts sh[code] applied), by
// the whole block of kBlock threads: thread tid takes halo slots tid,
// tid + kBlock, ...; hidx holds the tile's slots as j | code << 24.  All of
// the thread's index loads, then all of its position loads are issued before
// its LDS stores.  The caller synchronises the block afterwards.
template <int D, int CAP>
__device__ __forceinline__ void stage_halo(const TileHdr& hdr, const uint32_t* hidx,
                                           const double (*sh)[4], const double4* P, double* hx,
                                           double* hy, double* hz) {
  const int tid = threadIdx.x;
  constexpr int SU = (CAP + kBlock - 1) / kBlock;
  uint32_t e[SU];
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int h = tid + u * kBlock;
    e[u] = h < hdr.halo ? hidx[h] : 0u;
  }
  double4 p[SU];
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int h = tid + u * kBlock;
    if (h < hdr.halo) p[u] = P[e[u] & kIdxMask];
  }
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int h = tid + u * kBlock;
    if (h < hdr.halo) {
      const int code = (int)(e[u] >> kCodeShift);
      hx[h] = p[u].x + sh[code][0];
      hy[h] = p[u].y + sh[code][1];
      if (D == 3) hz[h] = p[u].z + sh[code][2];
    }
  }
}

// stage_halo with this thread's compact-halo entries already loaded: ent[u]
// holds slot tid + u kBlock of the tile's compact halo (any value past the
// halo size, which is not read).
template <int D, int CAP>
__device__ __forceinline__ void stage_halo_from(const TileHdr& hdr, const uint32_t* ent,
                                                const double (*sh)[4], const double4* P, double* hx,
                                                double* hy, double* hz) {
  const int tid = threadIdx.x;
  constexpr int SU = (CAP + kBlock - 1) / kBlock;
  double4 p[SU];
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int h = tid + u * kBlock;
    if (h < hdr.halo) p[u] = P[ent[u] & kIdxMask];
  }
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int h = tid + u * kBlock;
    if (h < hdr.halo) {
      const int code = (int)(ent[u] >> kCodeShift);
      hx[h] = p[u].x + sh[code][0];
      hy[h] = p[u].y + sh[code][1];
      if (D == 3) hz[h] = p[u].z + sh[code][2];
    }
  }
}

// Atom range of segment s of row `row` (rows cut into m segments).
__device__ __forceinline__ void segment(const int* nc, int m, const int32_t* cs, int t, int& a0,
                                        int& a1, int& cy, int& cz) {
  const int row = t / m, s = t % m;
  cy = row % nc[1];
  cz = row / nc[1];
  const int c0 = (cz * nc[1] + cy) * nc[0];
  const int r0 = cs[c0], len = cs[c0 + nc[0]] - r0;
  a0 = r0 + (int)(((int64_t)s * len) / m);
  a1 = r0 + (int)(((int64_t)(s + 1) * len) / m);
}

}  // namespace aqs
