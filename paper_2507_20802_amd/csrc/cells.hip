// cells.hip -- cell binning by counting sort and Verlet neighbour lists on
// gfx950, for the slots whose lists the host rebuilds.
//
// Steps (one launch each, all on the context stream):
//   grid   copy the host-chosen cell grid into the slot state
//   zero   clear per-cell counts
//   bin    fractional coordinates s = H^-1 r (Eq. 1 box); wrap r into the
//          primary cell (r -= H floor(s)); cell index; integer atomic count
//   scan   exclusive scan of the counts per slot (one workgroup per slot)
//   scat   place each atom in its cell (order inside a cell arbitrary)
//   sort   sort each cell by atom id (gives a deterministic order)
//   perm   gather positions, velocities, ids into scratch in the new order
//   back   copy back; inverse permutation
//   list   per force tile (tiles.h): its segment and halo run table, then
//          per atom the 3^dim neighbouring cells, keeping every image pair
//          within rc_ab + skin; tiles with an LDS halo get the packed list
//          (16-bit byte offsets 8 h of the neighbour's halo slot h), the
//          others the word list (j | image code << 24); engine.h
//   done   reset the validity bound of each rebuilt slot
// Integer atomics only; the result does not depend on their order.
#include <hip/hip_runtime.h>

#include "cellgeom.h"
#include "kernels.h"
#include "tiles.h"

namespace aqs {

namespace {

// grid per slot: nc0, nc1, nc2, tile width, tiles, list mode
__global__ void k_rb_grid(RebuildArgs a, const int32_t* nc3) {
  const int r = blockIdx.x;
  if (threadIdx.x == 0 && r < a.nreps) {
    State* st = a.state + a.reps[r];
    const int32_t* q = nc3 + kGridInts * r;
    st->nc[0] = q[0];
    st->nc[1] = q[1];
    st->nc[2] = q[2];
    st->tiles_x = q[3];
    st->ntiles = q[4];
    st->list_mode = q[5];
  }
}

__global__ void k_rb_zero(RebuildArgs a) {
  const int rep = a.reps[blockIdx.y];
  const Geom& g = a.geom[rep];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= g.cell_cap) {
    a.cell_count[g.cell_off + c] = 0;
    a.cell_start[g.cell_off + c] = 0;
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_rb_bin(RebuildArgs a) {
  const int2 bt = a.blocks[blockIdx.x];
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  const State* st = a.state + bt.x;
  const int li = bt.y * kBlock + threadIdx.x;
  if (li >= g.n) return;
  const int64_t gi = g.atom_off + li;
  const Box b = box_at(g, st->k);
  double4 p = a.pos4[gi];
  double s[3];
  frac(b, p.x, p.y, (D == 3) ? p.z : 0.0, s);
  const double nx = floor(s[0]), ny = floor(s[1]), nz = (D == 3) ? floor(s[2]) : 0.0;
  if (nx != 0.0 || ny != 0.0 || nz != 0.0) {
    // back into the box: r -= H n
    p.x -= nx * b.h00 + ny * b.h01;
    p.y -= (b.h10 == 0.0) ? ny * b.h11 : nx * b.h10 + ny * b.h11;
    if (D == 3) p.z -= nz * b.h22;
    a.pos4[gi] = p;
    if (a.alt4) {
      double4 q = a.alt4[gi];
      q.x -= nx * b.h00 + ny * b.h01;
      q.y -= (b.h10 == 0.0) ? ny * b.h11 : nx * b.h10 + ny * b.h11;
      if (D == 3) q.z -= nz * b.h22;
      a.alt4[gi] = q;
    }
  }
  int c3[3];
  const int nc[3] = {st->nc[0], st->nc[1], st->nc[2]};
  const int c = cell_of_pos<D>(b, nc, p, c3);
  a.cell_of[gi] = c;
  atomicAdd(a.cell_count + g.cell_off + c, 1);
}

__global__ __launch_bounds__(1024) void k_rb_scan(RebuildArgs a) {
  const int rep = a.reps[blockIdx.x];
  const Geom g = a.geom[rep];
  const State* st = a.state + rep;
  const int ncell = st->nc[0] * st->nc[1] * st->nc[2];
  __shared__ int part[1024];
  const int T = blockDim.x;
  const int per = (ncell + T - 1) / T;
  const int c0 = threadIdx.x * per, c1 = min(ncell, c0 + per);
  int sum = 0;
  for (int c = c0; c < c1; ++c) sum += a.cell_count[g.cell_off + c];
  part[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums (integers: exact)
  for (int off = 1; off < T; off <<= 1) {
    const int v = (threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = (threadIdx.x == 0) ? 0 : part[threadIdx.x - 1];
  for (int c = c0; c < c1; ++c) {
    const int n = a.cell_count[g.cell_off + c];
    a.cell_start[g.cell_off + c] = run;
    a.cell_count[g.cell_off + c] = run;  // becomes the scatter cursor
    run += n;
  }
  if (threadIdx.x == T - 1) a.cell_start[g.cell_off + ncell] = part[T - 1];
}

__global__ __launch_bounds__(kBlock) void k_rb_scatter(RebuildArgs a) {
  const int2 bt = a.blocks[blockIdx.x];
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  const int li = bt.y * kBlock + threadIdx.x;
  if (li >= g.n) return;
  const int64_t gi = g.atom_off + li;
  const int c = a.cell_of[gi];
  const int pos = atomicAdd(a.cell_count + g.cell_off + c, 1);
  a.order[g.atom_off + pos] = li;
}

// Sort each cell by atom id: one wavefront per cell (4 cells per block).
// Each atom's new place is its rank among the cell's ids (ids are distinct),
// counted against a copy of the cell in LDS.  Cells larger than kSortCap
// (only possible for very dense random starts) fall back to an insertion
// sort by one lane.
constexpr int kSortCap = 192;

__global__ __launch_bounds__(256) void k_rb_sort(RebuildArgs a) {
  const int rep = a.reps[blockIdx.y];
  const Geom g = a.geom[rep];
  const State* st = a.state + rep;
  const int ncell = st->nc[0] * st->nc[1] * st->nc[2];
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int c = blockIdx.x * 4 + wv;
  __shared__ int keys[4][kSortCap];
  __shared__ int vals[4][kSortCap];
  int b = 0, n = 0;
  int32_t* o = a.order + g.atom_off;
  const int32_t* id = a.id + g.atom_off;
  if (c < ncell) {
    b = a.cell_start[g.cell_off + c];
    n = a.cell_start[g.cell_off + c + 1] - b;
  }
  const bool fits = n <= kSortCap;
  if (fits)
    for (int k = lane; k < n; k += kWave) {
      const int v = o[b + k];
      vals[wv][k] = v;
      keys[wv][k] = id[v];
    }
  __syncthreads();
  if (fits) {
    for (int k = lane; k < n; k += kWave) {
      const int key = keys[wv][k];
      int r = 0;
      for (int q = 0; q < n; ++q) r += (keys[wv][q] < key) ? 1 : 0;
      o[b + r] = vals[wv][k];
    }
  } else if (lane == 0) {
    for (int i = b + 1; i < b + n; ++i) {  // insertion sort by atom id
      const int v = o[i];
      const int key = id[v];
      int j = i - 1;
      while (j >= b && id[o[j]] > key) {
        o[j + 1] = o[j];
        --j;
      }
      o[j + 1] = v;
    }
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_rb_perm(RebuildArgs a) {
  const int2 bt = a.blocks[blockIdx.x];
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  const int li = bt.y * kBlock + threadIdx.x;
  if (li >= g.n) return;
  const int64_t gi = g.atom_off + li;
  const int64_t go = g.atom_off + a.order[gi];
  a.tpos4[gi] = a.pos4[go];
  a.tvx[gi] = a.vx[go];
  a.tvy[gi] = a.vy[go];
  if (D == 3) a.tvz[gi] = a.vz[go];
  a.tid_[gi] = a.id[go];
  if (a.dlx) {
    a.tdlx[gi] = a.dlx[go];
    a.tdly[gi] = a.dly[go];
    if (D == 3) a.tdlz[gi] = a.dlz[go];
  }
  if (a.alt4) a.talt4[gi] = a.alt4[go];
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_rb_back(RebuildArgs a) {
  const int2 bt = a.blocks[blockIdx.x];
  if (bt.x < 0) return;
  const Geom g = a.geom[bt.x];
  const int li = bt.y * kBlock + threadIdx.x;
  if (li >= g.n) return;
  const int64_t gi = g.atom_off + li;
  a.pos4[gi] = a.tpos4[gi];
  a.xref4[gi] = a.tpos4[gi];
  a.vx[gi] = a.tvx[gi];
  a.vy[gi] = a.tvy[gi];
  if (D == 3) a.vz[gi] = a.tvz[gi];
  const int32_t aid = a.tid_[gi];
  a.id[gi] = aid;
  a.inv[g.atom_off + aid] = li;
  if (a.dlx) {
    a.dlx[gi] = a.tdlx[gi];
    a.dly[gi] = a.tdly[gi];
    if (D == 3) a.dlz[gi] = a.tdlz[gi];
  }
  if (a.alt4) a.alt4[gi] = a.talt4[gi];
}

// Neighbour lists, one block per force tile (tiles.h): the tile's segment
// and candidate runs are computed here; the scan marks every candidate some
// list names, the marked candidates numbered in order form the compact halo
// (stored for the force kernel as j | code << 24), and each entry is the
// byte offset of its compact halo slot (or, for a tile whose compact halo
// does not fit in LDS, the neighbour's global index and image code).
template <int D>
__global__ __launch_bounds__(kBlock) void k_rb_list(RebuildArgs a) {
  const int2 bt = a.tiles[blockIdx.x];
  if (bt.x < 0) return;
  const State* st = a.state + bt.x;
  if (bt.y >= st->ntiles) return;
  const Geom g = a.geom[bt.x];
  const Box bx = box_at(g, st->k);
  const int nc[3] = {st->nc[0], st->nc[1], st->nc[2]};
  const int32_t* cs = a.cell_start + g.cell_off;
  const double4* P = a.pos4 + g.atom_off;
  const int tid = threadIdx.x;
  __shared__ TileRun runs[kRuns];
  __shared__ int s_cx0, s_cx1, s_cand, s_lds, s_ncand;
  __shared__ uint32_t s_bits[kHaloWords];   // candidates named by some list
  __shared__ int s_pre[kHaloWords];          // marked candidates before each word
  int a0, a1, cy, cz;
  segment(nc, st->tiles_x, cs, bt.y, a0, a1, cy, cz);
  if (tid == 0) {
    int c3[3];
    s_cx0 = 0;
    s_cx1 = 0;
    if (a1 > a0) {
      cell_of_pos<D>(bx, nc, P[a0], c3);
      s_cx0 = c3[0];
      cell_of_pos<D>(bx, nc, P[a1 - 1], c3);
      s_cx1 = c3[0];
    }
  }
  __syncthreads();
  if (tid < kRuns) runs[tid] = make_run<D>(tid, s_cx0, s_cx1, cy, cz, nc, cs);
  for (int w = tid; w < kHaloWords; w += kBlock) s_bits[w] = 0u;
  __syncthreads();
  constexpr int CAP = (D == 3) ? kHaloCap3 : kHaloCap2;
  const int64_t tix = g.tile_off + bt.y;
  const int nt = a1 - a0;
  const bool sortable = nt <= kTileSort;
  if (tid == 0) {
    int off = 0;
    for (int r = 0; r < kRuns; ++r) {
      runs[r].off = off;
      off += runs[r].count;
    }
    s_ncand = off;
    s_cand = (st->list_mode == 0 && off <= 32 * kHaloWords && sortable) ? 1 : 0;
  }
  __syncthreads();
  // cand: entries hold candidate numbers during the scan and become compact
  // halo offsets (or global entries) below
  const bool cand = s_cand != 0;
  const int ncand = s_ncand;
  // Work area: the staged candidates during the scan, the staged list rows
  // in the final pass.  Candidates are FP32 offsets from the tile's first
  // atom with their image shift applied, and their types.
  __shared__ __align__(16) unsigned char s_work[kCandCap * (4 * D + 1)];
  float* s_cx = reinterpret_cast<float*>(s_work);
  float* s_cy = s_cx + kCandCap;
  float* s_cz = s_cy + kCandCap;                      // 3D only
  uint8_t* s_ct = reinterpret_cast<uint8_t*>(s_cx + D * kCandCap);
  __shared__ int s_cnt0[kTileSort];   // list counts in tile order
  const double4 ref = nt > 0 ? P[a0] : make_double4(0.0, 0.0, 0.0, 0.0);
  if (cand) {
    for (int hc = tid; hc < ncand; hc += kBlock) {
      int r = 0;
      while (r < kRuns - 1 && !(hc >= runs[r].off && hc < runs[r].off + runs[r].count)) ++r;
      const double4 pj = P[runs[r].src + (hc - runs[r].off)];
      double sft[3];
      code_shift(runs[r].code, bx, sft);
      s_cx[hc] = (float)((pj.x + sft[0]) - ref.x);
      s_cy[hc] = (float)((pj.y + sft[1]) - ref.y);
      if (D == 3) s_cz[hc] = (float)((pj.z + sft[2]) - ref.z);
      s_ct[hc] = (uint8_t)pj.w;
    }
    __syncthreads();
  }
  for (int li = a0 + tid; li < a1; li += kBlock) {
    const int64_t gi = g.atom_off + li;
    const double4 pi = P[li];
    const int tyi = (int)pi.w;
    double rl2[2];
    float rl2f[2];
    for (int b = 0; b < 2; ++b) {
      const double rc = sqrt(a.pp[2 * tyi + b].rc2) + a.skin;
      rl2[b] = rc * rc;
      rl2f[b] = (float)((rc + kListMargin) * (rc + kListMargin));
    }
    const float pix = (float)(pi.x - ref.x), piy = (float)(pi.y - ref.y),
                piz = (D == 3) ? (float)(pi.z - ref.z) : 0.0f;
    int c3[3];
    cell_of_pos<D>(bx, nc, pi, c3);
    uint32_t* L = a.nbl + g.nb_off + li;
    int na = 0, nb = 0;   // A neighbours from row 0 up, B neighbours from row max_nb - 1 down
    bool over = false;
    const int zlo = (D == 3) ? -1 : 0, zhi = (D == 3) ? 1 : 0;
    for (int dz = zlo; dz <= zhi; ++dz) {
      int cz2 = c3[2] + dz, iz = 0;
      if (D == 3) {
        if (cz2 < 0) { cz2 += nc[2]; iz = -1; }
        else if (cz2 >= nc[2]) { cz2 -= nc[2]; iz = 1; }
      }
      for (int dy = -1; dy <= 1; ++dy) {
        int cy2 = c3[1] + dy, iy = 0;
        if (cy2 < 0) { cy2 += nc[1]; iy = -1; }
        else if (cy2 >= nc[1]) { cy2 -= nc[1]; iy = 1; }
        for (int dx = -1; dx <= 1; ++dx) {
          int cx = c3[0] + dx, ix = 0;
          if (cx < 0) { cx += nc[0]; ix = -1; }
          else if (cx >= nc[0]) { cx -= nc[0]; ix = 1; }
          const int code = (ix + 1) + 3 * (iy + 1) + 9 * (iz + 1);
          const TileRun& rr = runs[run_of(c3[0], dx, dy, dz, nc[0])];
          double sh[3];
          box_shift(bx, ix, iy, iz, sh);
          const double sx = sh[0], sy = sh[1], sz = sh[2];
          const int c = (cz2 * nc[1] + cy2) * nc[0] + cx;
          const int jb = cs[c], je = cs[c + 1];
          if (cand) {
            // staged candidates, FP32 with the margin
            const int hb = rr.off + (jb - rr.src);
            for (int q = 0; q < je - jb; ++q) {
              if (jb + q == li && code == 13) continue;
              const int hc = hb + q;
              const float fx = s_cx[hc] - pix, fy = s_cy[hc] - piy;
              const float fz = (D == 3) ? s_cz[hc] - piz : 0.0f;
              const int tj = s_ct[hc];
              if (fx * fx + fy * fy + fz * fz < rl2f[tj]) {
                atomicOr(&s_bits[hc >> 5], 1u << (hc & 31));
                if (na + nb < a.max_nb) {
                  const int row = (tj == 0) ? na : a.max_nb - 1 - nb;
                  L[(int64_t)row * g.npad] = (uint32_t)hc;
                } else {
                  over = true;
                }
                if (tj == 0) ++na; else ++nb;
              }
            }
            continue;
          }
          for (int j = jb; j < je; ++j) {
            if (j == li && code == 13) continue;
            const double4 pj = P[j];
            const double ddx = (pj.x - pi.x) + sx;
            const double ddy = (pj.y - pi.y) + sy;
            const double ddz = (D == 3) ? (pj.z - pi.z) + sz : 0.0;
            const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (r2 < rl2[(int)pj.w]) {
              const uint32_t hc = (uint32_t)(rr.off + (j - rr.src));
              const uint32_t ent = cand ? hc : ((uint32_t)j | ((uint32_t)code << kCodeShift));
              if (cand) atomicOr(&s_bits[hc >> 5], 1u << (hc & 31));
              if (na + nb < a.max_nb) {
                const int row = (pj.w == 0.0) ? na : a.max_nb - 1 - nb;
                L[(int64_t)row * g.npad] = ent;
              } else {
                over = true;
              }
              if (pj.w == 0.0) ++na; else ++nb;
            }
          }
        }
      }
    }
    a.nbc[gi] = na | (nb << 16);
    if (sortable) s_cnt0[li - a0] = na | (nb << 16);
    // a tile with an LDS halo also needs the atom's A and B groups of the
    // packed list to fit side by side
    const int G = a.max_nb / kGroup;
    if (cand && (na + kGroup - 1) / kGroup + (nb + kGroup - 1) / kGroup > G) over = true;
    if (over) atomicMax(a.overflow, na + nb);
  }
  __syncthreads();
  // compact halo: the marked candidates, numbered in candidate order
  __shared__ int s_max[2];
  if (tid < kHaloWords) s_pre[tid] = __popc(s_bits[tid]);
  if (tid == 0) {
    s_max[0] = 0;
    s_max[1] = 0;
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int w = 0; w < kHaloWords; ++w) {
      const int c = s_pre[w];
      s_pre[w] = acc;
      acc += c;
    }
    // LDS halo slot CAP - 1 is the force kernel's far fill slot
    const bool lds = cand && acc < CAP;
    s_lds = lds ? 1 : 0;
    TileHdr h;
    h.a0 = a0;
    h.a1 = a1;
    h.pad_ = 0;
    h.halo = lds ? acc : -1;
    a.thdr[tix] = h;
  }
  __syncthreads();
  const bool lds = s_lds != 0;
  // Walk order.  The consumers of a tile with an LDS halo walk its atoms by
  // decreasing list length (ties by position), so the lanes of a wavefront
  // have lists of similar length: tord[a0 + k] is the k-th atom, and its
  // packed list and count sit in column a0 + k, so a wavefront still reads
  // consecutive list words.  Other tiles keep their atoms in tile order.
  __shared__ int s_src[kTileSort];
  int32_t* nbc = a.nbc + g.atom_off;
  for (int li = a0 + tid; li < a1; li += kBlock) {
    const int ci = (nbc[li] & 0xffff) + (nbc[li] >> 16);
    int rank = li - a0;
    if (lds) {   // lds implies cand, so the tile is sortable and s_cnt0 is set
      rank = 0;
      for (int k = 0; k < nt; ++k) {
        const int cj = (s_cnt0[k] & 0xffff) + (s_cnt0[k] >> 16);
        rank += (cj > ci || (cj == ci && k < li - a0)) ? 1 : 0;
      }
      s_src[rank] = li - a0;
    }
    a.tord[g.atom_off + a0 + rank] = li;
    atomicMax(&s_max[0], nbc[li] & 0xffff);
    atomicMax(&s_max[1], nbc[li] >> 16);
  }
  if (lds) {
    uint32_t* hx = a.hidx + tix * CAP;
    for (int hc = tid; hc < ncand; hc += kBlock) {
      const uint32_t w = s_bits[hc >> 5], bit = 1u << (hc & 31);
      if (!(w & bit)) continue;
      int r = 0;
      while (r < kRuns - 1 && !(hc >= runs[r].off && hc < runs[r].off + runs[r].count)) ++r;
      hx[s_pre[hc >> 5] + __popc(w & (bit - 1u))] =
          (uint32_t)(runs[r].src + (hc - runs[r].off)) | ((uint32_t)runs[r].code << kCodeShift);
    }
  }
  __syncthreads();
  if (!cand) return;   // entries are already j | code, columns in tile order
  if (!lds) {
    // the compact halo does not fit: candidate numbers -> j | code in place,
    // each atom's own rows only (its A and B rows never overlap)
    for (int li = a0 + tid; li < a1; li += kBlock) {
      const int c = nbc[li], na = c & 0xffff, nb = c >> 16;
      uint32_t* L = a.nbl + g.nb_off + li;
      for (int q = 0; q < na + nb; ++q) {
        const int64_t row = q < na ? q : a.max_nb - 1 - (q - na);
        const int hc = min((int)L[row * g.npad], ncand - 1);
        int r = 0;
        while (r < kRuns - 1 && !(hc >= runs[r].off && hc < runs[r].off + runs[r].count)) ++r;
        L[row * g.npad] =
            (uint32_t)(runs[r].src + (hc - runs[r].off)) | ((uint32_t)runs[r].code << kCodeShift);
      }
    }
    return;
  }
  // Tile with an LDS halo: counts in walk order, then the packed list.  The
  // word list keeps the scan's candidate numbers (original columns); each
  // pass stages kGroup rows per group row of the tile's atoms in LDS and
  // writes the groups of every atom in its walk-order column, entry =
  // byte offset 8 h of the candidate's compact halo slot h, the last group
  // of a segment padded with the far fill slot.
  __shared__ int s_cnt[kTileSort];
  uint32_t* s_stage = reinterpret_cast<uint32_t*>(s_work);   // the candidates are dead now
  for (int k = tid; k < nt; k += kBlock) s_cnt[k] = s_cnt0[s_src[k]];
  __syncthreads();
  for (int k = tid; k < nt; k += kBlock) nbc[a0 + k] = s_cnt[k];
  const int G = a.max_nb / kGroup;
  const int rows_a = min(s_max[0], a.max_nb), rows_b = min(s_max[1], a.max_nb);
  const int ga = (rows_a + kGroup - 1) / kGroup, gb = (rows_b + kGroup - 1) / kGroup;
  const int ng = ga + gb;
  const int ntc = max(nt, 1);
  const int pg = max(1, kRowStage / (kGroup * ntc));
  const uint32_t* Lt = a.nbl + g.nb_off + a0;
  uint2* Pk = a.nbp + g.nb_off / kGroup + a0;
  const uint32_t fill = 8u * (uint32_t)(CAP - 1);
  auto halo_offset = [&](uint32_t hc) -> uint32_t {
    hc = min(hc, (uint32_t)(ncand - 1));
    const uint32_t w = s_bits[hc >> 5], bit = 1u << (hc & 31);
    return 8u * (uint32_t)(s_pre[hc >> 5] + __popc(w & (bit - 1u)));
  };
  for (int g0 = 0; g0 < ng; g0 += pg) {
    const int cnt = min(pg, ng - g0);
    const int ne = cnt * kGroup * nt;
    for (int e = tid; e < ne; e += kBlock) {
      const int gq = g0 + e / (kGroup * nt), i = (e / nt) % kGroup, col = e % nt;
      const bool isa = gq < ga;
      const int q = kGroup * (isa ? gq : gq - ga) + i;
      const bool ok = q < (isa ? rows_a : rows_b);
      s_stage[e] = ok ? Lt[(int64_t)(isa ? q : a.max_nb - 1 - q) * g.npad + col] : 0u;
    }
    __syncthreads();
    for (int e = tid; e < cnt * nt; e += kBlock) {
      const int gq = g0 + e / nt, k = e % nt;
      const bool isa = gq < ga;
      const int gs = isa ? gq : gq - ga;   // group of the atom's segment
      const int nk = isa ? (s_cnt[k] & 0xffff) : (s_cnt[k] >> 16);
      if (kGroup * gs >= nk) continue;     // not one of this atom's groups
      const int src = s_src[k];
      const int base = (e / nt) * kGroup * nt;
      uint32_t o[kGroup];
#pragma unroll
      for (int i = 0; i < kGroup; ++i)
        o[i] = (kGroup * gs + i < nk) ? halo_offset(s_stage[base + i * nt + src]) : fill;
      Pk[(int64_t)(isa ? gs : G - 1 - gs) * g.npad + k] =
          make_uint2(o[0] | (o[1] << 16), o[2] | (o[3] << 16));
    }
    __syncthreads();
  }
}

__global__ void k_rb_done(RebuildArgs a) {
  const int rep = a.reps[blockIdx.x];
  const Geom& g = a.geom[rep];
  State* st = a.state + rep;
  for (int b = threadIdx.x; b < g.nblocks; b += blockDim.x) a.upart[g.block0 + b] = 0.0;
  if (threadIdx.x == 0) {
    st->ubound = 0.0;
    st->gamma_build = strain_of(st->k, g.dgamma);
    st->k_build = st->k;
    if (a.resume && st->phase == PH_REBUILD)
      st->phase = (st->resume_phase == PH_LPLAIN || st->resume_phase == PH_LMOVE ||
                   st->resume_phase == PH_LREVERT || st->resume_phase == PH_CG)
                      ? st->resume_phase
                      : PH_FIRE;
  }
}

}  // namespace

void launch_rebuild(const RebuildArgs& a, int32_t max_cells_per_slot, hipStream_t s,
                    const int32_t* nc3_dev) {
  if (a.nreps <= 0 || a.nblk <= 0) return;
  const int cb = (max_cells_per_slot + 1 + 255) / 256;
  hipLaunchKernelGGL(k_rb_grid, dim3(a.nreps), dim3(64), 0, s, a, nc3_dev);
  hipLaunchKernelGGL(k_rb_zero, dim3(cb, a.nreps), dim3(256), 0, s, a);
  if (a.dim == 3) {
    hipLaunchKernelGGL(k_rb_bin<3>, dim3(a.nblk), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_rb_bin<2>, dim3(a.nblk), dim3(kBlock), 0, s, a);
  }
  hipLaunchKernelGGL(k_rb_scan, dim3(a.nreps), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_rb_scatter, dim3(a.nblk), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_rb_sort, dim3((max_cells_per_slot + 3) / 4, a.nreps), dim3(256), 0, s, a);
  if (a.dim == 3) {
    hipLaunchKernelGGL(k_rb_perm<3>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_rb_back<3>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_rb_list<3>, dim3(a.ntile_blk), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_rb_perm<2>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_rb_back<2>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_rb_list<2>, dim3(a.ntile_blk), dim3(kBlock), 0, s, a);
  }
  hipLaunchKernelGGL(k_rb_done, dim3(a.nreps), dim3(256), 0, s, a);
}

}  // namespace aqs
