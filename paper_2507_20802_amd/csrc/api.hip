// api.hip -- host side of the AQS engine: workspace layout, slot state,
// launch tables, the minimisation driver loop and the C ABI of include/aqs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "aqs.h"
#include "kernels.h"
#include "learned.h"
#include "linear.h"

using namespace aqs;

namespace {

thread_local std::string g_err;

aqs_status fail(aqs_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(AQS_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));             \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

double rc_max_of(const aqs_potential* p) {
  double m = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) m = std::max(m, p->rc_factor * p->sigma[a][b]);
  return m;
}

// A launch table places each entry on an XCD by the round-robin rule of
// kXcds (engine.h).
constexpr uint32_t kAllXcds = (1u << kXcds) - 1u;

// force tiles hold about fill x a block's atom lanes (tuning.tile_fill)
constexpr double kFillDefault = 0.9, kFillMin = 0.5, kFillMax = 2.0;

struct Tune {
  double skin;
  int max_nb, block_iters, use_graph, log_cap, tpa;
  int live_blocks;   // batch force blocks per CU beside a critical chain (0: no limit)
  int live_xcds;     // XCDs reserved for the critical chain of a live round (0: none)
  double tile_fill;  // force-tile atoms per block's atom lanes
  int force_waves;   // force kernel occupancy target (waves per SIMD): 4 or 5
  int live_duty;     // live rounds: the batch runs one block in live_duty (1: every block)
  int lin_max_cg;    // linear-response start: updates of the solve at most
  double lin_tol;    // ... stop at |r| <= lin_tol |f(x0)|
  double lin_probe;  // ... probe length of the Hessian-vector products
};

Tune resolve(const aqs_potential* pot, const aqs_tuning* t) {
  Tune r;
  r.skin = (t && t->skin > 0.0) ? t->skin : 0.3;
  r.max_nb = (t && t->max_neighbors > 0) ? t->max_neighbors : (pot->dim == 3 ? 192 : 64);
  // the packed list holds max_nb / kGroup groups, shared by up to kMaxTPA lanes
  r.max_nb = (r.max_nb + kListAlign - 1) / kListAlign * kListAlign;
  // even: a block's iterations alternate the state buffers and end in the home one
  r.block_iters = (t && t->block_iters > 0) ? (t->block_iters + 1) / 2 * 2 : 32;
  r.use_graph = t ? t->use_graph : 0;
  r.log_cap = ((t && t->max_chain_steps > 0) ? t->max_chain_steps : 1024) + 1;
  const int tp = t ? t->threads_per_atom : 0;
  r.tpa = (tp == 1 || tp == 2 || tp == 4 || tp == 8) ? tp : 2;
  const int lb = t ? t->live_batch_blocks : 0;
  r.live_blocks = lb < 0 ? 0 : (lb == 0 ? 3 : std::min(lb, 4));
  const int lx = t ? t->live_xcds : 0;
  r.live_xcds = std::max(0, std::min(lx, kXcds - 1));
  const double tf = t ? t->tile_fill : 0.0;
  r.tile_fill = tf > 0.0 ? std::max(kFillMin, std::min(tf, kFillMax)) : kFillDefault;
  r.force_waves = (t && t->force_waves == 4) ? 4 : 5;
  r.live_duty = 1;
  r.lin_max_cg = 50;
  r.lin_tol = 1e-3;
  r.lin_probe = 1e-5;
  return r;
}

// Cells per axis of a slot's grid: the perpendicular width of the deformed
// box along each Bravais vector (|det| over the length of the other edge in
// the (x, y) block) divided by the list cutoff, at least 3 (the 3^dim stencil).
void cell_grid(int dim, const Box& b, double rl, int* nc) {
  if (b.h10 == 0.0) {
    const double wx = b.h00 * b.h11 / std::sqrt(b.h11 * b.h11 + b.h01 * b.h01);
    nc[0] = (int)std::floor(wx / rl);
    nc[1] = (int)std::floor(b.h11 / rl);
  } else {
    const double det = std::fabs(b.h00 * b.h11 - b.h01 * b.h10);
    nc[0] = (int)std::floor(det / std::sqrt(b.h01 * b.h01 + b.h11 * b.h11) / rl);
    nc[1] = (int)std::floor(det / std::sqrt(b.h00 * b.h00 + b.h10 * b.h10) / rl);
  }
  nc[2] = dim == 3 ? (int)std::floor(b.h22 / rl) : 1;
}

// Segments per cell row of the force tiles: about `fill` times a block's
// atom lanes (kBlock / threads_per_atom) per segment on average.
int segments_per_row(int n, int rows, int tpa, double fill) {
  const int per = kBlock / tpa;
  const double mean_row = (double)n / rows;
  return std::max(1, (int)std::ceil(mean_row / (fill * per)));
}

// Entries of a launch table over n items spread over any subset of the XCDs
// (at most kXcds (n + 1)).
size_t table_cap(int64_t n) { return (size_t)kXcds * ((size_t)n + 1); }

struct Layout {
  size_t total = 0;
  size_t o_geom, o_state, o_state2, o_cgst, o_cgst2, o_pos4, o_v[3], o_f[3], o_id, o_inv, o_nbc, o_nbl, o_nbp, o_fpart, o_upart, o_upart2,
      o_log, o_ccount, o_cstart, o_cellof, o_order, o_tpos4, o_tv[3], o_tid, o_tbl[2],
      o_tbl2[2], o_reps[2], o_nc3[2], o_overflow[2], o_dg, o_red, o_dl[3], o_tdl[3], o_alt4, o_talt4, o_evals, o_xref4, o_ftbl[2], o_ttbl[2], o_thdr, o_hidx, o_sel[2],
      o_zbuf, o_lpart, o_mlp, o_mlpw, o_ltbl[2], o_lftbl[2], o_lsel[2], o_tord, o_lin;
  int64_t atoms = 0;      // padded atoms over all slots
  int64_t nb_entries = 0;
  int32_t blocks = 0;
  int32_t cells = 0;      // sum of (cell_cap + 1)
  int32_t tiles = 0;      // sum of tile_cap
  int32_t max_cells = 0;
  std::vector<Geom> geom;
};

aqs_status make_layout(const aqs_potential* pot, const Tune& tn, int n_rep, const int32_t* n_atoms,
                       const double* box_len, const double* dgamma, Layout& lo) {
  const int dim = pot->dim;
  if (dim != 2 && dim != 3) return fail(AQS_EINVAL, "dim must be 2 or 3 (got %d)", dim);
  if (n_rep <= 0) return fail(AQS_EINVAL, "n_rep must be positive");
  const double rl = rc_max_of(pot) + tn.skin;
  lo.geom.resize(n_rep);
  int64_t atom_off = 0, nb_off = 0;
  int32_t block0 = 0, cell_off = 0;
  for (int r = 0; r < n_rep; ++r) {
    const int n = n_atoms[r];
    if (n <= 0 || n > (int)kIdxMask) return fail(AQS_EINVAL, "slot %d: bad atom count %d", r, n);
    Geom& g = lo.geom[r];
    g.n = n;
    g.npad = (int)align_up((size_t)n, kBlock);
    g.atom_off = atom_off;
    g.nb_off = nb_off;
    g.block0 = block0;
    g.nblocks = g.npad / kBlock;
    for (int a = 0; a < 3; ++a) g.L[a] = (a < dim) ? box_len[r * dim + a] : 1.0;
    g.dgamma = dgamma ? dgamma[r] : 0.0;
    g.dgamma_y = 0.0;
    int nc[3];
    cell_grid(dim, box_at(g, 0), rl, nc);
    for (int a = 0; a < dim; ++a)
      if (nc[a] < 3)
        return fail(AQS_EINVAL,
                    "slot %d: box edge %g too small; need >= 3 (rc_max + skin) = %g", r,
                    g.L[a], 3.0 * rl);
    // the force kernel addresses a slot's list with 32-bit byte offsets
    if ((int64_t)g.npad * tn.max_nb >= (int64_t(1) << 30))
      return fail(AQS_ECAPACITY, "slot %d: neighbour list of %d atoms x %d entries exceeds 2^30 words",
                  r, g.npad, tn.max_nb);
    g.cell_cap = nc[0] * nc[1] * nc[2];
    g.cell_off = cell_off;
    // force tiles: rows x segments; rows are fixed by the grid in y, z
    g.tile_off = lo.tiles;
    g.tile_cap = nc[1] * nc[2] * segments_per_row(n, nc[1] * nc[2], kMaxTPA, kFillMin);
    lo.tiles += g.tile_cap;
    lo.max_cells = std::max(lo.max_cells, g.cell_cap);
    atom_off += g.npad;
    nb_off += (int64_t)g.npad * tn.max_nb;
    block0 += g.nblocks;
    cell_off += g.cell_cap + 1;
  }
  lo.atoms = atom_off;
  lo.nb_entries = nb_off;
  lo.blocks = block0;
  lo.cells = cell_off;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t A = (size_t)lo.atoms;
  lo.o_geom = take(sizeof(Geom) * n_rep);
  lo.o_state = take(sizeof(State) * n_rep);
  lo.o_state2 = take(sizeof(State) * n_rep);
  lo.o_cgst = take(sizeof(CgState) * n_rep);
  lo.o_cgst2 = take(sizeof(CgState) * n_rep);
  lo.o_pos4 = take(sizeof(double4) * A);
  for (int a = 0; a < 3; ++a) lo.o_v[a] = take(sizeof(double) * A);
  for (int a = 0; a < 3; ++a) lo.o_f[a] = take(sizeof(double) * A);
  lo.o_id = take(sizeof(int32_t) * A);
  lo.o_inv = take(sizeof(int32_t) * A);
  lo.o_nbc = take(sizeof(int32_t) * A);
  lo.o_nbl = take(sizeof(uint32_t) * (size_t)lo.nb_entries);
  lo.o_nbp = take(sizeof(uint16_t) * (size_t)lo.nb_entries);
  lo.o_fpart = take(sizeof(double) * kForceParts * (size_t)lo.tiles);
  lo.o_thdr = take(sizeof(TileHdr) * (size_t)lo.tiles);
  lo.o_hidx = take(sizeof(uint32_t) * (size_t)halo_cap(dim) * (size_t)lo.tiles);
  lo.o_upart = take(sizeof(double) * (size_t)lo.blocks);
  lo.o_upart2 = take(sizeof(double) * (size_t)lo.blocks);
  lo.o_log = take(sizeof(StepRecord) * (size_t)n_rep * tn.log_cap);
  lo.o_ccount = take(sizeof(int32_t) * (size_t)lo.cells);
  lo.o_cstart = take(sizeof(int32_t) * (size_t)lo.cells);
  lo.o_cellof = take(sizeof(int32_t) * A);
  lo.o_order = take(sizeof(int32_t) * A);
  lo.o_tpos4 = take(sizeof(double4) * A);
  for (int a = 0; a < 3; ++a) lo.o_tv[a] = take(sizeof(double) * A);
  lo.o_tid = take(sizeof(int32_t) * A);
  for (int l = 0; l < 2; ++l) {   // per driver lane
    lo.o_tbl[l] = take(sizeof(int2) * table_cap(lo.blocks));
    lo.o_tbl2[l] = take(sizeof(int2) * table_cap(lo.blocks));
    lo.o_reps[l] = take(sizeof(int32_t) * n_rep);
    lo.o_sel[l] = take(sizeof(int32_t) * n_rep);
    lo.o_nc3[l] = take(sizeof(int32_t) * kGridInts * n_rep);
    lo.o_overflow[l] = take(sizeof(int32_t));
    lo.o_ftbl[l] = take(sizeof(int2) * table_cap(lo.tiles));
    lo.o_ttbl[l] = take(sizeof(int2) * table_cap(lo.tiles));
    lo.o_ltbl[l] = take(sizeof(int2) * table_cap(lo.blocks));
    lo.o_lftbl[l] = take(sizeof(int2) * table_cap(lo.tiles));
    lo.o_lsel[l] = take(sizeof(int32_t) * n_rep);
  }
  lo.o_dg = take(sizeof(double) * 4 * n_rep);
  lo.o_red = take(sizeof(double) * 10 * ((size_t)lo.blocks + 8));
  for (int a = 0; a < 3; ++a) lo.o_dl[a] = take(sizeof(double) * A);
  for (int a = 0; a < 3; ++a) lo.o_tdl[a] = take(sizeof(double) * A);
  lo.o_alt4 = take(sizeof(double4) * A);
  lo.o_talt4 = take(sizeof(double4) * A);
  lo.o_evals = take(2 * sizeof(unsigned long long));   // all evaluations, timed ones
  lo.o_xref4 = take(sizeof(double4) * A);
  lo.o_zbuf = take(sizeof(uint16_t) * kFeat * A);
  lo.o_lpart = take(sizeof(double) * kLearnParts * ((size_t)lo.blocks + 8));
  lo.o_mlp = take(sizeof(MlpDev));
  lo.o_mlpw = take(sizeof(float) * kNumParams);
  lo.o_tord = take(sizeof(int32_t) * A);
  lo.o_lin = take(sizeof(LinState) * n_rep);
  lo.total = off;
  return AQS_OK;
}

template <class T>
T* at(char* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

// Launch state of one stream of the minimisation driver: launch tables
// (device, and pinned host staging) over its selection of slots, the rebuild
// and learned-start tables, its neighbour-list overflow flag and a captured
// iteration block.  Lane 0 runs on the context stream; lane 1, on a stream of
// its own, carries the critical chain of a live round (aqs_run_round).
struct Lane {
  hipStream_t s = nullptr;
  int2 *tbl = nullptr, *ftbl = nullptr, *tbl2 = nullptr, *ttbl = nullptr;
  int2 *ltbl = nullptr, *lftbl = nullptr;
  int32_t *sel_d = nullptr, *reps_d = nullptr, *nc3_d = nullptr, *lsel_d = nullptr;
  int32_t* overflow = nullptr;
  int2 *h_tbl = nullptr, *h_ftbl = nullptr, *h_tbl2 = nullptr, *h_ttbl = nullptr;
  int2 *h_ltbl = nullptr, *h_lftbl = nullptr;
  int32_t *h_sel = nullptr, *h_reps = nullptr, *h_nc3 = nullptr, *h_lsel = nullptr;
  int32_t* h_over = nullptr;
  std::vector<int32_t> cur_sel;    // slots of the current iteration tables
  int32_t cur_nblk = 0;
  int32_t cur_ntiles = 0;
  bool ftable_stale = false;       // a rebuild changed the tiles of the selection
  hipGraphExec_t gexec = nullptr;  // captured block of FIRE iterations (use_graph)
  int32_t g_iters = 0;
  int32_t g_pad = 0;               // its force launches' dynamic LDS
  bool in_flight = false;          // a block of iterations launched, not yet polled
  bool timed = false;              // ... with HIP events around its kernels
  bool prefetched = false;         // ... with its slots' states copied back behind it
  uint32_t xcd_mask = kAllXcds;    // XCDs its launch tables place blocks on
  std::vector<hipEvent_t> ev;      // the lane's timing events (4 per iteration)
};

}  // namespace

struct aqs_ctx {
  int dim = 0, n_rep = 0;
  aqs_potential pot{};
  Tune tn{};
  FireParams fire{};
  CgParams cg{};
  int32_t minimizer = kMinFire;   // of later minimisation calls
  bool live = false;              // a live round runs (aqs_run_round, live = 1)
  int32_t live_pad = -1;          // force_lds_pad of the live reservation (-1: not yet known)
  PairParams pp[4];
  double rc_max = 0.0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Layout lo;
  // device views
  Geom* d_geom;
  State* d_state;            // home buffer of the slot states (see IterArgs)
  State* d_state2;           // second buffer, written by odd iterations of a block
  CgState *cgst, *cgst2;
  double4* pos4;
  double *vx, *vy, *vz, *fx, *fy, *fz;
  int32_t *id, *inv, *nbc;
  uint32_t* nbl;
  uint2* nbp;
  double *fpart, *upart, *upart2;
  StepRecord* log;
  int32_t *ccount, *cstart, *cellof, *order, *tid;
  double4* tpos4;
  double *tvx, *tvy, *tvz;
  double *dg_d, *red;
  double *dlx, *dly, *dlz, *tdlx, *tdly, *tdlz;
  double4 *alt4, *talt4;
  unsigned long long* evals;
  double4* xref4;
  TileHdr* thdr;
  uint32_t* hidx;
  // learned start
  uint16_t* zbuf;
  double* lpart;
  MlpDev* mlp;
  float* mlpw;
  int32_t* tord;             // per tile: atoms by decreasing list length
  LinState* lin;             // linear-response start: per-slot solve scalars
  int64_t lin_evals = 0;     // atom evaluations of its solves (host count)
  int mlp_dim = 0;           // 0: no network loaded
  double rd[4], rd2[4], dirs[16][3];
  // host mirrors
  State* h_state = nullptr;  // pinned
  std::vector<char> loaded, dirty;
  std::vector<int32_t> tiles_now;  // force tiles of each slot's current grid
  // driver lanes (pinned staging: one use per synchronisation of the lane)
  Lane ln[2];
  double* h_dg = nullptr;
  // profiling
  int32_t prof_every = 0;
  int64_t block_count = 0;
  aqs_counters cnt{};
};

namespace {
bool lane_active(const aqs_ctx* c, const Lane& L);

// Dynamic LDS of the batch lane's force blocks: during a live round, while
// the critical chain runs on lane 1, the batch yields part of every compute
// unit to it (stream priorities and CU masks are not used).
int32_t batch_pad(aqs_ctx* c, const Lane& L) {
  if (!c->live || c->tn.live_blocks <= 0 || &L != &c->ln[0] || !lane_active(c, c->ln[1]))
    return 0;
  if (c->live_pad < 0) c->live_pad = force_lds_pad(c->dim, c->tn.tpa, c->tn.live_blocks);
  return c->live_pad;
}

IterArgs iter_args(aqs_ctx* c, const Lane& L) {
  IterArgs a{};
  a.blocks = L.tbl;
  a.ftiles = L.ftbl;
  a.sel = L.sel_d;
  a.nsel = (int32_t)L.cur_sel.size();
  a.tpa = c->tn.tpa;
  a.waves = c->tn.force_waves;
  a.lds_pad = batch_pad(c, L);
  a.prio = (c->live && &L == &c->ln[1]) ? 1 : 0;
  a.one_rep = -1;
  if (L.cur_sel.size() == 1 && L.xcd_mask == kAllXcds) {
    const int r = L.cur_sel[0];
    a.one_rep = r;
    a.one_ntiles = c->tiles_now[r];
    a.one_nblk = c->lo.geom[r].nblocks;
    a.one_tile0 = c->lo.geom[r].tile_off;
  }
  a.geom = c->d_geom;
  a.state = c->d_state;
  a.state_out = c->d_state2;
  a.state_home = c->d_state;
  a.pos4 = c->pos4;
  a.vx = c->vx; a.vy = c->vy; a.vz = c->vz;
  a.fx = c->fx; a.fy = c->fy; a.fz = c->fz;
  a.id = c->id; a.inv = c->inv;
  a.nbc = c->nbc; a.nbl = c->nbl; a.nbp = c->nbp;
  a.cell_start = c->cstart;
  a.thdr = c->thdr;
  a.hidx = c->hidx;
  a.tord = c->tord;
  a.fpart = c->fpart; a.upart = c->upart; a.upart_out = c->upart2;
  a.log = c->log; a.log_cap = c->tn.log_cap;
  a.max_nb = c->tn.max_nb;
  for (int t = 0; t < 4; ++t) a.pp[t] = c->pp[t];
  a.fire = c->fire;
  a.cg = c->cg;
  a.cgst = c->cgst;
  a.cgst_out = c->cgst2;
  a.minimizer = c->minimizer;
  a.skin = c->tn.skin;
  a.rc_max = c->rc_max;
  a.dlx = c->dlx; a.dly = c->dly; a.dlz = c->dlz;
  a.alt4 = c->alt4;
  a.gx = c->dlx; a.gy = c->dly; a.gz = c->dlz;
  a.evals = c->evals;
  a.xref4 = c->xref4;
  return a;
}

LearnArgs learn_args(aqs_ctx* c, const Lane& L, int mode, float* out = nullptr) {
  LearnArgs a{};
  a.blocks = L.tbl;
  a.ftiles = L.ftbl;
  a.thdr = c->thdr;
  a.hidx = c->hidx;
  a.nbl = c->nbl;
  a.nbp = c->nbp;
  a.nbc = c->nbc;
  a.tord = c->tord;
  a.max_nb = c->tn.max_nb;
  a.sel = L.sel_d;
  a.nsel = (int32_t)L.cur_sel.size();
  a.mode = mode;
  a.geom = c->d_geom;
  a.state = c->d_state;
  a.pos4 = c->pos4;
  a.vx = c->vx; a.vy = c->vy; a.vz = c->vz;
  a.id = c->id; a.inv = c->inv;
  a.cell_start = c->cstart;
  a.xref4 = c->xref4;
  a.upart = c->upart;
  a.lpart = c->lpart;
  a.zbuf = c->zbuf;
  a.dlx = c->dlx; a.dly = c->dly; a.dlz = c->dlz;
  a.alt4 = c->alt4;
  a.out = out;
  a.mlp = c->mlp;
  for (int t = 0; t < 4; ++t) {
    a.rd[t] = c->rd[t];
    a.rd2[t] = c->rd2[t];
  }
  for (int k = 0; k < 16; ++k)
    for (int q = 0; q < 3; ++q) a.dirs[k][q] = c->dirs[k][q];
  a.max_move = 0.1;
  return a;
}

std::vector<int2> make_table(aqs_ctx* c, const std::vector<int32_t>& sel, uint32_t xcds,
                             int per_block = 1);
std::vector<int2> make_tile_table(aqs_ctx* c, const std::vector<int32_t>& sel, uint32_t xcds,
                                  bool global = true);

// Learned (or extrapolated) start of the slots waiting in PH_LDESC (known
// from the last state read-back): descriptors and network, or the
// extrapolation; plain start and the checks, with launch tables over exactly
// those slots.
// The lane's start tables over the slots ls: 256-atom blocks, force tiles
// of their current grids, the slots.  Returns the block and tile counts.
// Uses the lane's pinned staging: the lane must be synchronised.
aqs_status start_tables(aqs_ctx* c, Lane& L, const std::vector<int32_t>& ls, int32_t* nblk,
                        int32_t* ntiles) {
  const std::vector<int2> tb = make_table(c, ls, L.xcd_mask);
  const std::vector<int2> ft = make_tile_table(c, ls, L.xcd_mask);
  std::copy(tb.begin(), tb.end(), L.h_ltbl);
  std::copy(ft.begin(), ft.end(), L.h_lftbl);
  std::copy(ls.begin(), ls.end(), L.h_lsel);
  HIPCHK(hipMemcpyAsync(L.ltbl, L.h_ltbl, sizeof(int2) * tb.size(), hipMemcpyHostToDevice, L.s));
  HIPCHK(hipMemcpyAsync(L.lftbl, L.h_lftbl, sizeof(int2) * ft.size(), hipMemcpyHostToDevice, L.s));
  HIPCHK(hipMemcpyAsync(L.lsel_d, L.h_lsel, sizeof(int32_t) * ls.size(), hipMemcpyHostToDevice,
                        L.s));
  *nblk = (int32_t)tb.size();
  *ntiles = (int32_t)ft.size();
  return AQS_OK;
}

aqs_status learned_group(aqs_ctx* c, Lane& L, const std::vector<int32_t>& ls, bool extrap) {
  int32_t nb = 0, nt = 0;
  aqs_status st = start_tables(c, L, ls, &nb, &nt);
  if (st) return st;
  LearnArgs la = learn_args(c, L, 0);
  la.blocks = L.ltbl;
  la.ftiles = L.lftbl;
  la.sel = L.lsel_d;
  la.nsel = (int32_t)ls.size();
  if (extrap) {
    launch_lextrap(la, nb, c->dim, L.s);
  } else {
    launch_ldesc(la, nt, c->dim, L.s);
    launch_lmlp(la, nb, c->dim, L.s);
  }
  launch_lctl(la, L.s);
  HIPCHK(hipGetLastError());
  return AQS_OK;
}

aqs_status rebuild(aqs_ctx* c, Lane& L, const std::vector<int32_t>& sel, bool in_loop,
                   int list_mode);
aqs_status pull_slots(aqs_ctx* c, Lane& L, const std::vector<int32_t>& slots);
aqs_status set_table(aqs_ctx* c, Lane& L, const std::vector<int32_t>& sel);
IterArgs iter_args(aqs_ctx* c, const Lane& L);

// Linear-response start (Eqs. 7-8, linear.hip) of the slots waiting in
// PH_LDESC: the plain start and k + 1 (the extrapolation kernels with u = 0),
// a list rebuild where a probe could leave the list's validity, then the
// conjugate-gradient solve of H u = f(x0), driven from here: per update two
// probes of the forces and three vector kernels, the stop flags read back
// every few updates; then u in the start's displacement arrays and the
// pre-check, phase PH_LPLAIN.
aqs_status linear_group(aqs_ctx* c, Lane& L, const std::vector<int32_t>& ls) {
  int32_t nb = 0, nt = 0;
  aqs_status st = start_tables(c, L, ls, &nb, &nt);
  if (st) return st;
  {
    LearnArgs la = learn_args(c, L, 0);
    la.blocks = L.ltbl;
    la.ftiles = L.lftbl;
    la.sel = L.lsel_d;
    la.nsel = (int32_t)ls.size();
    launch_lextrap(la, nb, c->dim, L.s);
    launch_lctl(la, L.s);
    HIPCHK(hipGetLastError());
  }
  // the probes move atoms by at most lin_probe beyond the plain start: the
  // list test of the control with that margin, else a rebuild now
  st = pull_slots(c, L, ls);
  if (st) return st;
  std::vector<int32_t> stale;
  std::vector<std::vector<double>> up(ls.size());
  for (size_t i = 0; i < ls.size(); ++i) {
    const Geom& g = c->lo.geom[ls[i]];
    up[i].resize(g.nblocks);
    HIPCHK(hipMemcpyAsync(up[i].data(), c->upart + g.block0, sizeof(double) * g.nblocks,
                          hipMemcpyDeviceToHost, L.s));
  }
  HIPCHK(hipStreamSynchronize(L.s));
  for (size_t i = 0; i < ls.size(); ++i) {
    const int r = ls[i];
    const Geom& g = c->lo.geom[r];
    double ub = 0.0;
    for (double u : up[i]) ub = std::max(ub, u);
    ub += c->tn.lin_probe;
    const State& s = c->h_state[r];
    bool valid;
    if (g.dgamma_y == 0.0) {
      const double gd = std::fabs(strain_of(s.k, g.dgamma) - s.gamma_build);
      valid = gd * c->rc_max + 2.0 * (1.0 + gd) * ub < c->tn.skin;
    } else {
      valid = inverse_strain_norm(g, s.k, s.k_build) * (c->rc_max + 2.0 * ub) < c->rc_max + c->tn.skin;
    }
    if (!valid) stale.push_back(r);
  }
  if (!stale.empty()) {
    st = rebuild(c, L, stale, false, 0);
    if (st) return st;
    if (L.ftable_stale) {   // the lane's own tables, as after a rebuild in the loop
      const std::vector<int32_t> keep = L.cur_sel;
      st = set_table(c, L, keep);
      if (st) return st;
    }
    HIPCHK(hipStreamSynchronize(L.s));
    st = start_tables(c, L, ls, &nb, &nt);   // the rebuilt grids' tiles
    if (st) return st;
  }
  LinArgs a{};
  a.blocks = L.ltbl;
  a.sel = L.lsel_d;
  a.nsel = (int32_t)ls.size();
  a.geom = c->d_geom;
  a.state = c->d_state;
  a.lin = c->lin;
  a.pos4 = c->pos4;
  a.x0 = c->alt4;
  a.fx = c->fx; a.fy = c->fy; a.fz = c->fz;
  a.ux = c->dlx; a.uy = c->dly; a.uz = c->dlz;
  a.px = c->vx; a.py = c->vy; a.pz = c->vz;
  a.r4 = c->tpos4;
  a.hx = c->tvx; a.hy = c->tvy; a.hz = c->tvz;
  a.part = c->lpart;
  a.probe = c->tn.lin_probe;
  a.tol = c->tn.lin_tol;
  a.max_move = 0.1;
  IterArgs fa = iter_args(c, L);
  fa.ftiles = L.lftbl;
  fa.one_rep = -1;
  launch_lin_begin(a, L.s);
  launch_force(fa, nt, c->dim, L.s);   // f(x0)
  launch_lin_init(a, nb, c->dim, L.s);
  launch_lin_start(a, L.s);
  int64_t pairs = 0;
  for (int it = 0; it < c->tn.lin_max_cg; ++it) {
    a.it = it;
    launch_lin_probe(a, 1, nb, c->dim, L.s);
    launch_force(fa, nt, c->dim, L.s);
    launch_lin_probe(a, -1, nb, c->dim, L.s);
    launch_force(fa, nt, c->dim, L.s);
    launch_lin_hp(a, nb, c->dim, L.s);
    launch_lin_update(a, nb, c->dim, L.s);
    launch_lin_direction(a, nb, c->dim, L.s);
    HIPCHK(hipGetLastError());
    ++pairs;
    if ((it + 1) % 4 == 0 && it + 1 < c->tn.lin_max_cg) {   // stop once every solve has
      std::vector<LinState> cur(ls.size());
      for (size_t i = 0; i < ls.size(); ++i)
        HIPCHK(hipMemcpyAsync(&cur[i], c->lin + ls[i], sizeof(LinState), hipMemcpyDeviceToHost, L.s));
      HIPCHK(hipStreamSynchronize(L.s));
      bool all = true;
      for (const LinState& q : cur) all = all && q.done;
      if (all) break;
    }
  }
  launch_lin_finish(a, nb, c->dim, L.s);
  HIPCHK(hipGetLastError());
  // evaluations for the counters: f(x0) and two per Hessian-vector product
  std::vector<LinState> fin(ls.size());
  for (size_t i = 0; i < ls.size(); ++i)
    HIPCHK(hipMemcpyAsync(&fin[i], c->lin + ls[i], sizeof(LinState), hipMemcpyDeviceToHost, L.s));
  HIPCHK(hipStreamSynchronize(L.s));
  for (size_t i = 0; i < ls.size(); ++i)
    c->lin_evals += (int64_t)c->lo.geom[ls[i]].n * (1 + 2 * (int64_t)fin[i].probes);
  c->cnt.force_launches += 1 + 2 * pairs;
  return AQS_OK;
}

// Launch table of the items `logical` on the XCDs of the mask: position b
// (hardware block b, on XCD b mod 8) holds an item only if that XCD is in
// the mask, and each of those XCDs gets a contiguous run of items, so
// neighbouring tiles share its L2; other positions hold slot -1 (the block
// exits at once).
std::vector<int2> xcd_table(const std::vector<int2>& logical, uint32_t xcds) {
  int rank[kXcds], nx = 0;
  for (int x = 0; x < kXcds; ++x) rank[x] = ((xcds >> x) & 1u) ? nx++ : -1;
  if (nx == 0) {   // no XCD named: all of them
    for (int x = 0; x < kXcds; ++x) rank[x] = x;
    nx = kXcds;
  }
  const size_t nb = logical.size();
  const size_t per = (nb + nx - 1) / nx;
  std::vector<int2> tbl(per * kXcds, make_int2(-1, 0));
  for (size_t b = 0; b < tbl.size(); ++b) {
    const int xr = rank[b % kXcds];
    if (xr < 0) continue;
    const size_t lk = (size_t)xr * per + b / kXcds;
    if (lk < nb) tbl[b] = logical[lk];
  }
  return tbl;
}

// Launch table over the 256-atom blocks of the given slots.
std::vector<int2> make_table(aqs_ctx* c, const std::vector<int32_t>& sel, uint32_t xcds,
                             int per_block) {
  std::vector<int2> logical;
  for (int r : sel) {
    const Geom& g = c->lo.geom[r];
    for (int b = 0; b < g.nblocks * per_block; ++b) logical.push_back(make_int2(r, b));
  }
  return xcd_table(logical, xcds);
}

// Launch table over the force tiles of the given slots' current grids:
// entries (slot, global tile index tile_off + t) for the force and
// descriptor kernels, (slot, t) for the list builder (global = false).
std::vector<int2> make_tile_table(aqs_ctx* c, const std::vector<int32_t>& sel, uint32_t xcds,
                                  bool global) {
  std::vector<int2> logical;
  for (int r : sel) {
    const int off = global ? c->lo.geom[r].tile_off : 0;
    for (int t = 0; t < c->tiles_now[r]; ++t) logical.push_back(make_int2(r, off + t));
  }
  return xcd_table(logical, xcds);
}

// Host copy of every slot's state (and lane 0's overflow flag), on the
// context stream.
aqs_status pull_state(aqs_ctx* c) {
  Lane& L = c->ln[0];
  HIPCHK(hipMemcpyAsync(c->h_state, c->d_state, sizeof(State) * c->n_rep, hipMemcpyDeviceToHost,
                        L.s));
  HIPCHK(hipMemcpyAsync(L.h_over, L.overflow, sizeof(int32_t), hipMemcpyDeviceToHost, L.s));
  HIPCHK(hipStreamSynchronize(L.s));
  return AQS_OK;
}

// Host copy of the states of the given slots (and the lane's overflow flag)
// on the lane's stream: the only states that lane's kernels write.
aqs_status pull_slots(aqs_ctx* c, Lane& L, const std::vector<int32_t>& slots) {
  for (int r : slots)
    HIPCHK(hipMemcpyAsync(c->h_state + r, c->d_state + r, sizeof(State), hipMemcpyDeviceToHost,
                          L.s));
  HIPCHK(hipMemcpyAsync(L.h_over, L.overflow, sizeof(int32_t), hipMemcpyDeviceToHost, L.s));
  HIPCHK(hipStreamSynchronize(L.s));
  return AQS_OK;
}

aqs_status push_slots(aqs_ctx* c, Lane& L, const std::vector<int32_t>& slots) {
  for (int r : slots)
    HIPCHK(hipMemcpyAsync(c->d_state + r, c->h_state + r, sizeof(State), hipMemcpyHostToDevice,
                          L.s));
  HIPCHK(hipStreamSynchronize(L.s));
  return AQS_OK;
}

// Neighbour-list overflow recorded by a rebuild of the lane since the last check.
aqs_status check_overflow(aqs_ctx* c, Lane& L) {
  if (*L.h_over > 0) {
    const int over = *L.h_over;
    *L.h_over = 0;
    HIPCHK(hipMemsetAsync(L.overflow, 0, sizeof(int32_t), L.s));
    HIPCHK(hipStreamSynchronize(L.s));
    return fail(AQS_ECAPACITY, "neighbour list overflow: an atom has %d neighbours, capacity %d",
                over, c->tn.max_nb);
  }
  return AQS_OK;
}

aqs_status push_state(aqs_ctx* c) {
  HIPCHK(hipMemcpyAsync(c->d_state, c->h_state, sizeof(State) * c->n_rep, hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return AQS_OK;
}

Box box_of(aqs_ctx* c, int r, int64_t k) { return box_at(c->lo.geom[r], k); }

// Rebuild cell order and neighbour lists of the given slots (positions as
// they are on the device; h_state must be current).
aqs_status rebuild(aqs_ctx* c, Lane& L, const std::vector<int32_t>& sel, bool in_loop = false,
                   int list_mode = 0) {
  if (sel.empty()) return AQS_OK;
  const double rl = c->rc_max + c->tn.skin;
  std::vector<int32_t> nc3(kGridInts * sel.size());
  for (size_t i = 0; i < sel.size(); ++i) {
    const int r = sel[i];
    const Geom& g = c->lo.geom[r];
    int nc[3];
    cell_grid(c->dim, box_of(c, r, c->h_state[r].k), rl, nc);
    for (int a = 0; a < c->dim; ++a)
      if (nc[a] < 3)
        return fail(AQS_EINVAL, "slot %d: sheared box too thin for the cell stencil", r);
    if (nc[0] * nc[1] * nc[2] > g.cell_cap)
      return fail(AQS_EINVAL, "slot %d: cell grid exceeds capacity", r);
    int32_t* q = &nc3[kGridInts * i];
    for (int a = 0; a < 3; ++a) q[a] = nc[a];
    q[3] = segments_per_row(g.n, nc[1] * nc[2], c->tn.tpa, c->tn.tile_fill);
    q[4] = q[3] * nc[1] * nc[2];
    if (q[4] > g.tile_cap) return fail(AQS_EINVAL, "slot %d: force tiles exceed capacity", r);
    q[5] = list_mode;
    if (c->tiles_now[r] != q[4]) {
      c->tiles_now[r] = q[4];
      if (std::find(L.cur_sel.begin(), L.cur_sel.end(), r) != L.cur_sel.end())
        L.ftable_stale = true;
    }
  }
  std::vector<int2> tbl = make_table(c, sel, L.xcd_mask);
  std::vector<int2> ttbl = make_tile_table(c, sel, L.xcd_mask, false);
  std::copy(tbl.begin(), tbl.end(), L.h_tbl2);
  std::copy(ttbl.begin(), ttbl.end(), L.h_ttbl);
  HIPCHK(hipMemcpyAsync(L.ttbl, L.h_ttbl, sizeof(int2) * ttbl.size(), hipMemcpyHostToDevice, L.s));
  std::copy(sel.begin(), sel.end(), L.h_reps);
  std::copy(nc3.begin(), nc3.end(), L.h_nc3);
  HIPCHK(hipMemcpyAsync(L.tbl2, L.h_tbl2, sizeof(int2) * tbl.size(), hipMemcpyHostToDevice, L.s));
  HIPCHK(hipMemcpyAsync(L.reps_d, L.h_reps, sizeof(int32_t) * sel.size(), hipMemcpyHostToDevice,
                        L.s));
  HIPCHK(hipMemcpyAsync(L.nc3_d, L.h_nc3, sizeof(int32_t) * nc3.size(), hipMemcpyHostToDevice,
                        L.s));
  RebuildArgs a{};
  a.blocks = L.tbl2;
  a.nblk = (int32_t)tbl.size();
  a.tiles = L.ttbl;
  a.ntile_blk = (int32_t)ttbl.size();
  a.reps = L.reps_d;
  a.nreps = (int32_t)sel.size();
  a.geom = c->d_geom;
  a.state = c->d_state;
  a.pos4 = c->pos4;
  a.xref4 = c->xref4;
  a.vx = c->vx; a.vy = c->vy; a.vz = c->vz;
  a.id = c->id; a.inv = c->inv;
  a.nbc = c->nbc; a.nbl = c->nbl; a.nbp = c->nbp;
  a.thdr = c->thdr; a.hidx = c->hidx; a.tord = c->tord;
  a.cell_count = c->ccount; a.cell_start = c->cstart; a.cell_of = c->cellof; a.order = c->order;
  a.tpos4 = c->tpos4; a.tvx = c->tvx; a.tvy = c->tvy; a.tvz = c->tvz; a.tid_ = c->tid;
  a.upart = c->upart;
  a.overflow = L.overflow;
  for (int t = 0; t < 4; ++t) a.pp[t] = c->pp[t];
  a.skin = c->tn.skin;
  a.max_nb = c->tn.max_nb;
  a.dim = c->dim;
  a.resume = in_loop ? 1 : 0;
  a.dlx = c->dlx; a.dly = c->dly; a.dlz = c->dlz;
  a.tdlx = c->tdlx; a.tdly = c->tdly; a.tdlz = c->tdlz;
  a.alt4 = c->alt4; a.talt4 = c->talt4;
  launch_rebuild(a, c->lo.max_cells, L.s, L.nc3_d);
  HIPCHK(hipGetLastError());
  ++c->cnt.rebuilds;
  for (int r : sel) c->dirty[r] = 0;
  // in the minimisation loop the next poll reads the overflow flag and the
  // state; elsewhere check now
  if (in_loop) return AQS_OK;
  aqs_status st = pull_state(c);
  if (st) return st;
  return check_overflow(c, L);
}

aqs_status check_slot(aqs_ctx* c, int r) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (r < 0 || r >= c->n_rep) return fail(AQS_EINVAL, "slot %d out of range [0, %d)", r, c->n_rep);
  if (!c->loaded[r]) return fail(AQS_ESTATE, "slot %d has no configuration", r);
  return AQS_OK;
}

void drop_graph(Lane& L) {
  if (L.gexec) (void)hipGraphExecDestroy(L.gexec);
  L.gexec = nullptr;
  L.g_iters = 0;
}

// The arguments of the next iteration: the in and out buffers of the state,
// conjugate-gradient state and displacement partials swapped.
IterArgs swapped(const IterArgs& a) {
  IterArgs b = a;
  std::swap(b.state, b.state_out);
  std::swap(b.cgst, b.cgst_out);
  std::swap(b.upart, b.upart_out);
  return b;
}

// M FIRE iterations (force, then control and move, per iteration; M even, so
// the block ends with everything in the home buffers) on the lane's stream:
// replayed from a captured hipGraph when use_graph is set and the stream can
// be captured, else launched directly.  The captured graph holds kernel
// launches only (no memset nodes).
aqs_status launch_block(aqs_ctx* c, Lane& L, const IterArgs& a, int M) {
  const IterArgs ab[2] = {a, swapped(a)};
  if (c->tn.use_graph && L.s != nullptr) {
    if (!L.gexec || L.g_iters != M || L.g_pad != a.lds_pad) {
      drop_graph(L);
      L.g_pad = a.lds_pad;
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(L.s, hipStreamCaptureModeThreadLocal));
      for (int it = 0; it < M; ++it) {
        launch_force(ab[it & 1], L.cur_ntiles, c->dim, L.s);
        launch_step(ab[it & 1], L.cur_nblk, c->dim, L.s);
      }
      const hipError_t ce = hipStreamEndCapture(L.s, &graph);
      if (ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(AQS_EHIP, "capturing the iteration block failed: %s", hipGetErrorString(ce));
      }
      const hipError_t ie = hipGraphInstantiate(&L.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        L.gexec = nullptr;
        return fail(AQS_EHIP, "instantiating the iteration block failed: %s", hipGetErrorString(ie));
      }
      L.g_iters = M;
    }
    HIPCHK(hipGraphLaunch(L.gexec, L.s));
    return AQS_OK;
  }
  for (int it = 0; it < M; ++it) {
    launch_force(ab[it & 1], L.cur_ntiles, c->dim, L.s);
    launch_step(ab[it & 1], L.cur_nblk, c->dim, L.s);
  }
  return AQS_OK;
}

aqs_status set_table(aqs_ctx* c, Lane& L, const std::vector<int32_t>& sel) {
  std::vector<int2> tbl = make_table(c, sel, L.xcd_mask);
  std::vector<int2> ftbl = make_tile_table(c, sel, L.xcd_mask);
  std::copy(tbl.begin(), tbl.end(), L.h_tbl);
  std::copy(ftbl.begin(), ftbl.end(), L.h_ftbl);
  HIPCHK(hipMemcpyAsync(L.tbl, L.h_tbl, sizeof(int2) * tbl.size(), hipMemcpyHostToDevice, L.s));
  HIPCHK(hipMemcpyAsync(L.ftbl, L.h_ftbl, sizeof(int2) * ftbl.size(), hipMemcpyHostToDevice, L.s));
  std::copy(sel.begin(), sel.end(), L.h_sel);
  HIPCHK(hipMemcpyAsync(L.sel_d, L.h_sel, sizeof(int32_t) * sel.size(), hipMemcpyHostToDevice,
                        L.s));
  HIPCHK(hipStreamSynchronize(L.s));
  drop_graph(L);   // the captured launches bake in the table sizes
  L.cur_sel = sel;
  L.cur_nblk = (int32_t)tbl.size();
  L.cur_ntiles = (int32_t)ftbl.size();
  L.ftable_stale = false;
  return AQS_OK;
}

void free_pinned(aqs_ctx* c) {
  std::vector<void*> ps = {c->h_state, c->h_dg};
  for (Lane& L : c->ln) {
    for (void* p : {(void*)L.h_tbl, (void*)L.h_ftbl, (void*)L.h_tbl2, (void*)L.h_ttbl,
                    (void*)L.h_ltbl, (void*)L.h_lftbl, (void*)L.h_sel, (void*)L.h_reps,
                    (void*)L.h_nc3, (void*)L.h_lsel, (void*)L.h_over})
      ps.push_back(p);
    L.h_tbl = L.h_ftbl = L.h_tbl2 = L.h_ttbl = L.h_ltbl = L.h_lftbl = nullptr;
    L.h_sel = L.h_reps = L.h_nc3 = L.h_lsel = L.h_over = nullptr;
  }
  for (void* p : ps)
    if (p) (void)hipHostFree(p);
  c->h_state = nullptr;
  c->h_dg = nullptr;
}

void reset_minimizer(aqs_ctx* c, State& s);

// Checks and initial state of the chains of a minimisation call: slot rep
// r = sel[i] gets its FIRE state reset, n_steps[i] fine steps and the
// snapshot slot snap_dst[i]; lists are rebuilt.
aqs_status start_chains(aqs_ctx* c, const std::vector<int32_t>& sel, int32_t start_mode,
                        const int32_t* n_steps, const int32_t* snap_dst) {
  if (start_mode != AQS_START_PLAIN && !predicted_start_mode(start_mode))
    return fail(AQS_EINVAL, "unknown start mode %d", start_mode);
  if (start_mode == AQS_START_LEARNED && c->mlp_dim != c->dim)
    return fail(AQS_ESTATE, "the learned start needs a network (aqs_learned_load)");
  const int n_sel = (int)sel.size();
  std::vector<char> seen(c->n_rep, 0);
  for (int i = 0; i < n_sel; ++i) {
    aqs_status st = check_slot(c, sel[i]);
    if (st) return st;
    if (seen[sel[i]]) return fail(AQS_EINVAL, "slot %d selected twice", sel[i]);
    seen[sel[i]] = 1;
    const int ns = n_steps ? n_steps[i] : 0;
    if (ns < 0 || ns + 1 > c->tn.log_cap)
      return fail(AQS_ECAPACITY, "n_steps %d outside [0, %d]", ns, c->tn.log_cap - 1);
    if (snap_dst && snap_dst[i] >= 0) {
      const int d = snap_dst[i];
      if (d >= c->n_rep || c->lo.geom[d].n != c->lo.geom[sel[i]].n ||
          c->lo.geom[d].dgamma_y != c->lo.geom[sel[i]].dgamma_y ||
          c->lo.geom[d].dgamma != c->lo.geom[sel[i]].dgamma)
        return fail(AQS_EINVAL, "snapshot slot %d invalid for slot %d", d, sel[i]);
    }
  }
  if (snap_dst)
    for (int i = 0; i < n_sel; ++i)
      if (snap_dst[i] >= 0 && seen[snap_dst[i]])
        return fail(AQS_EINVAL, "snapshot slot %d is also being minimised", snap_dst[i]);
  aqs_status st = pull_state(c);
  if (st) return st;
  st = rebuild(c, c->ln[0], sel);
  if (st) return st;
  for (int i = 0; i < n_sel; ++i) {
    State& s = c->h_state[sel[i]];
    reset_minimizer(c, s);
    s.phase = (c->minimizer == kMinCG) ? PH_CG : PH_FIRE;
    s.status = -1;
    s.step = 0;
    s.n_steps = n_steps ? n_steps[i] : 0;
    s.snap_dst = snap_dst ? snap_dst[i] : -1;
    s.do_snap = 0;
    s.start_mode = start_mode;
    s.start_used = AQS_START_PLAIN;
    s.drops = 0;
    s.sxy_prev = 0.0;
  }
  return push_state(c);
}

bool lane_active(const aqs_ctx* c, const Lane& L) {
  for (int r : L.cur_sel)
    if (c->h_state[r].phase != PH_DONE) return true;
  return false;
}

// One block of block_iters FIRE iterations over the lane's selection (after
// the learned-start kernels for its slots waiting in PH_LDESC); with
// allow_timed, every prof_every-th block brackets its kernels with events.
aqs_status lane_launch(aqs_ctx* c, Lane& L, int32_t start_mode, bool allow_timed) {
  const bool timed = allow_timed && c->prof_every > 0 && (c->block_count % c->prof_every) == 0;
  const int M = c->tn.block_iters;
  if (timed) {
    while ((int)L.ev.size() < 4 * M) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      L.ev.push_back(e);
    }
  }
  if (predicted_start_mode(start_mode)) {
    // slots that finished a minimisation since the last read-back wait in
    // PH_LDESC: the predicted displacement and plain start for them now
    std::vector<int32_t> ls;
    for (int r : L.cur_sel)
      if (c->h_state[r].phase == PH_LDESC) ls.push_back(r);
    if (!ls.empty()) {
      aqs_status st = (start_mode == AQS_START_LINEAR)
                          ? linear_group(c, L, ls)
                          : learned_group(c, L, ls, start_mode == AQS_START_EXTRAPOLATED);
      if (st) return st;
    }
  }
  IterArgs a = iter_args(c, L);
  if (timed) a.tevals = c->evals + 1;   // atoms of the timed launches
  if (timed) {
    const IterArgs ab[2] = {a, swapped(a)};
    for (int it = 0; it < M; ++it) {
      // the force kernel's and the step kernel's own start and end times,
      // recorded with their dispatches (no marker packets in between)
      launch_force(ab[it & 1], L.cur_ntiles, c->dim, L.s, L.ev[4 * it + 0], L.ev[4 * it + 1]);
      launch_step(ab[it & 1], L.cur_nblk, c->dim, L.s, L.ev[4 * it + 2], L.ev[4 * it + 3]);
    }
  } else {
    aqs_status st = launch_block(c, L, a, M);
    if (st) return st;
  }
  HIPCHK(hipGetLastError());
  c->cnt.force_launches += M;
  if (allow_timed) ++c->block_count;
  L.prefetched = false;
  if (c->live) {
    // the lane's states and overflow flag copied back behind the block, so the
    // read-back after it costs no second round trip
    for (int r : L.cur_sel)
      HIPCHK(hipMemcpyAsync(c->h_state + r, c->d_state + r, sizeof(State), hipMemcpyDeviceToHost,
                            L.s));
    HIPCHK(hipMemcpyAsync(L.h_over, L.overflow, sizeof(int32_t), hipMemcpyDeviceToHost, L.s));
    L.prefetched = true;
  }
  L.in_flight = true;
  L.timed = timed;
  return AQS_OK;
}

// Read-back after a lane's block: its slots' states (all_states: every
// slot's, on the context stream), the overflow flag, event times; then the
// rebuilds its slots asked for (they resume on the device).  active: slots
// of the lane not yet done.
aqs_status lane_poll(aqs_ctx* c, Lane& L, bool all_states, int& active) {
  // (a prefetched lane's stream has completed: its copies are in host memory)
  aqs_status st = all_states ? pull_state(c) : (L.prefetched ? AQS_OK : pull_slots(c, L, L.cur_sel));
  if (st) return st;
  L.prefetched = false;
  st = check_overflow(c, L);
  if (st) return st;
  ++c->cnt.host_polls;
  L.in_flight = false;
  if (L.timed) {
    const int M = c->tn.block_iters;
    for (int it = 0; it < M; ++it) {
      float f = 0.f, u = 0.f;
      HIPCHK(hipEventElapsedTime(&f, L.ev[4 * it + 0], L.ev[4 * it + 1]));
      HIPCHK(hipEventElapsedTime(&u, L.ev[4 * it + 2], L.ev[4 * it + 3]));
      c->cnt.force_ms += f;
      c->cnt.update_ms += u;
    }
    c->cnt.force_timed += M;
    c->cnt.update_timed += M;
    L.timed = false;
  }
  std::vector<int32_t> rb;
  active = 0;
  for (int r : L.cur_sel) {
    const int ph = c->h_state[r].phase;
    if (ph == PH_REBUILD) rb.push_back(r);
    if (ph != PH_DONE) ++active;
  }
  if (!active) return AQS_OK;
  if (!rb.empty()) {
    st = rebuild(c, L, rb, true);
    if (st) return st;
  }
  // finished slots leave the launch tables (their blocks would only read
  // their phase and exit); a grid that changed its tile count also re-tables
  if (active < (int)L.cur_sel.size() || L.ftable_stale) {
    std::vector<int32_t> left;
    for (int r : L.cur_sel)
      if (c->h_state[r].phase != PH_DONE) left.push_back(r);
    return set_table(c, L, left);
  }
  return AQS_OK;
}

// Equality test of Eq. (20) between two idle slots, on the lane's stream
// (their states are read on that stream first).
aqs_status compare_slots(aqs_ctx* c, Lane& L, int32_t ra, int32_t rb, double delta_eq,
                         aqs_check* out) {
  const Geom& g = c->lo.geom[ra];
  aqs_status st = pull_slots(c, L, std::vector<int32_t>{ra, rb});
  if (st) return st;
  if (c->h_state[ra].k != c->h_state[rb].k)
    return fail(AQS_EINVAL, "slots %d and %d are at different strain indices (%lld vs %lld)", ra,
                rb, (long long)c->h_state[ra].k, (long long)c->h_state[rb].k);
  const int nb = (g.n + kBlock - 1) / kBlock;
  launch_compare(c->d_geom, ra, rb, g.n, c->pos4, c->inv, box_of(c, ra, c->h_state[ra].k), c->dim,
                 c->red, L.s);
  HIPCHK(hipGetLastError());
  std::vector<double> part(nb);
  HIPCHK(hipMemcpyAsync(part.data(), c->red, sizeof(double) * nb, hipMemcpyDeviceToHost, L.s));
  HIPCHK(hipStreamSynchronize(L.s));
  double m = 0.0;
  for (double v : part) m = std::max(m, v);
  out->decided = 1;
  out->equal = (m < delta_eq) ? 1 : 0;
  out->max_disp = m;
  out->de_per_atom = (c->h_state[ra].E - c->h_state[rb].E) / (double)g.n;
  return AQS_OK;
}

// End of a minimisation call (all lanes idle): slots back to PH_IDLE,
// snapshot slots marked loaded, records copied.  A cancelled chain keeps the
// records of its finished minimisations; its later ones read AQS_CANCELLED.
aqs_status finish_chains(aqs_ctx* c, const std::vector<int32_t>& sel, const int32_t* n_steps,
                         const int32_t* snap_dst, const std::vector<char>& cancelled,
                         aqs_step_record* records) {
  const int n_sel = (int)sel.size();
  int max_steps = 0;
  for (int i = 0; i < n_sel; ++i) max_steps = std::max(max_steps, n_steps ? n_steps[i] : 0);
  std::vector<int> done(n_sel);
  for (int i = 0; i < n_sel; ++i) {
    const int r = sel[i];
    // minimisations finished: 0 .. step, or 0 .. step - 1 when stopped early
    done[i] = cancelled[i] ? c->h_state[r].step : c->h_state[r].step + 1;
    c->h_state[r].phase = PH_IDLE;
    if (snap_dst && snap_dst[i] >= 0 && done[i] >= 1) {
      c->loaded[snap_dst[i]] = 1;
      c->dirty[snap_dst[i]] = 1;
    }
  }
  aqs_status st = push_state(c);
  if (st) return st;
  if (!records) return AQS_OK;
  const int stride = max_steps + 1;
  std::vector<StepRecord> tmp(c->tn.log_cap);
  for (int i = 0; i < n_sel; ++i) {
    const int r = sel[i];
    const int ns = done[i];
    if (ns > 0)
      HIPCHK(hipMemcpy(tmp.data(), c->log + (int64_t)r * c->tn.log_cap, sizeof(StepRecord) * ns,
                       hipMemcpyDeviceToHost));
    for (int s = 0; s < ns && s < stride; ++s) {
      aqs_step_record& o = records[(int64_t)i * stride + s];
      o.iters = tmp[s].iters;
      o.energy = tmp[s].energy;
      o.max_f = tmp[s].max_f;
      o.sigma_xy = tmp[s].sigma_xy;
      o.status = tmp[s].status;
      o.start = tmp[s].start;
    }
    if (cancelled[i]) {
      const int last = n_steps ? n_steps[i] : 0;
      for (int s = ns; s <= last && s < stride; ++s) {
        aqs_step_record& o = records[(int64_t)i * stride + s];
        o.iters = 0;
        o.energy = 0.0;
        o.max_f = 0.0;
        o.sigma_xy = 0.0;
        o.status = AQS_CANCELLED;
        o.start = AQS_START_PLAIN;
      }
    }
  }
  return AQS_OK;
}

void reset_minimizer(aqs_ctx* c, State& s) {
  s.dt = c->fire.dt0;
  s.alpha = c->fire.alpha0;
  s.cv = 1.0;
  s.cf = 0.0;
  s.npos = 0;
  s.nneg = 0;
  s.it = 0;
  s.restart = 0;
}

}  // namespace

extern "C" {

const char* aqs_last_error(void) { return g_err.c_str(); }

size_t aqs_workspace_bytes(const aqs_potential* pot, const aqs_tuning* tune, int32_t n_rep,
                           const int32_t* n_atoms, const double* box_len) {
  if (!pot || !n_atoms || !box_len) return 0;
  Layout lo;
  if (make_layout(pot, resolve(pot, tune), n_rep, n_atoms, box_len, nullptr, lo) != AQS_OK) return 0;
  return lo.total;
}

aqs_status aqs_create(const aqs_potential* pot, const aqs_fire_params* fire,
                      const aqs_tuning* tune, int32_t n_rep, const int32_t* n_atoms,
                      const double* box_len, const double* dgamma, void* workspace,
                      size_t workspace_bytes, void* stream, aqs_ctx** out) {
  if (!pot || !fire || !n_atoms || !box_len || !dgamma || !workspace || !out)
    return fail(AQS_EINVAL, "null argument to aqs_create");
  if (((uintptr_t)workspace) % 256 != 0) return fail(AQS_EINVAL, "workspace not 256-byte aligned");
  aqs_ctx* c = new aqs_ctx();
  c->dim = pot->dim;
  c->n_rep = n_rep;
  c->pot = *pot;
  c->tn = resolve(pot, tune);
  aqs_status st = make_layout(pot, c->tn, n_rep, n_atoms, box_len, dgamma, c->lo);
  if (st != AQS_OK) {
    delete c;
    return st;
  }
  if (workspace_bytes < c->lo.total) {
    size_t need = c->lo.total;
    delete c;
    return fail(AQS_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  }
  c->rc_max = rc_max_of(pot);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const double sig = pot->sigma[a][b], eps = pot->eps[a][b];
      const double rc = pot->rc_factor * sig;
      const double sc2 = (sig * sig) / (rc * rc);
      const double sc6 = sc2 * sc2 * sc2;
      PairParams& q = c->pp[2 * a + b];
      q.rc2 = rc * rc;
      q.sig2 = sig * sig;
      q.eps4 = 4.0 * eps;
      q.ucut = 4.0 * eps * (sc6 * sc6 - sc6);
      c->rd[2 * a + b] = rc;      // descriptor cutoff = the pair cutoff
      c->rd2[2 * a + b] = rc * rc;
    }
  // directions of the angular descriptors: 16 angles 2 pi k / 16 (2D),
  // the 16 points of a Fibonacci sphere (3D)
  for (int k = 0; k < 16; ++k) {
    if (pot->dim == 2) {
      const double an = 2.0 * M_PI * k / 16.0;
      c->dirs[k][0] = std::cos(an);
      c->dirs[k][1] = std::sin(an);
      c->dirs[k][2] = 0.0;
    } else {
      const double z = 1.0 - (2.0 * k + 1.0) / 16.0;
      const double rho = std::sqrt(1.0 - z * z);
      const double phi = (k * M_PI) * (3.0 - std::sqrt(5.0));
      c->dirs[k][0] = rho * std::cos(phi);
      c->dirs[k][1] = rho * std::sin(phi);
      c->dirs[k][2] = z;
    }
  }
  c->fire.dt0 = fire->dt0; c->fire.dt_max = fire->dt_max; c->fire.dt_min = fire->dt_min;
  c->fire.f_inc = fire->f_inc; c->fire.f_dec = fire->f_dec; c->fire.alpha0 = fire->alpha0;
  c->fire.f_alpha = fire->f_alpha; c->fire.dmax = fire->dmax; c->fire.ftol = fire->ftol;
  c->fire.n_delay = fire->n_delay; c->fire.n_neg_max = fire->n_neg_max;
  c->fire.initial_delay = fire->initial_delay; c->fire.max_iter = fire->max_iter;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  Layout& lo = c->lo;
  char* w = c->ws;
  c->d_geom = at<Geom>(w, lo.o_geom);
  c->d_state = at<State>(w, lo.o_state);
  c->d_state2 = at<State>(w, lo.o_state2);
  c->cgst = at<CgState>(w, lo.o_cgst);
  c->cgst2 = at<CgState>(w, lo.o_cgst2);
  c->pos4 = at<double4>(w, lo.o_pos4);
  c->vx = at<double>(w, lo.o_v[0]); c->vy = at<double>(w, lo.o_v[1]); c->vz = at<double>(w, lo.o_v[2]);
  c->fx = at<double>(w, lo.o_f[0]); c->fy = at<double>(w, lo.o_f[1]); c->fz = at<double>(w, lo.o_f[2]);
  c->id = at<int32_t>(w, lo.o_id);
  c->inv = at<int32_t>(w, lo.o_inv);
  c->nbc = at<int32_t>(w, lo.o_nbc);
  c->nbl = at<uint32_t>(w, lo.o_nbl);
  c->nbp = at<uint2>(w, lo.o_nbp);
  c->fpart = at<double>(w, lo.o_fpart);
  c->upart = at<double>(w, lo.o_upart);
  c->upart2 = at<double>(w, lo.o_upart2);
  c->log = at<StepRecord>(w, lo.o_log);
  c->ccount = at<int32_t>(w, lo.o_ccount);
  c->cstart = at<int32_t>(w, lo.o_cstart);
  c->cellof = at<int32_t>(w, lo.o_cellof);
  c->order = at<int32_t>(w, lo.o_order);
  c->tpos4 = at<double4>(w, lo.o_tpos4);
  c->tvx = at<double>(w, lo.o_tv[0]); c->tvy = at<double>(w, lo.o_tv[1]); c->tvz = at<double>(w, lo.o_tv[2]);
  c->tid = at<int32_t>(w, lo.o_tid);
  c->thdr = at<TileHdr>(w, lo.o_thdr);
  c->hidx = at<uint32_t>(w, lo.o_hidx);
  for (int l = 0; l < 2; ++l) {
    Lane& L = c->ln[l];
    L.tbl = at<int2>(w, lo.o_tbl[l]);
    L.tbl2 = at<int2>(w, lo.o_tbl2[l]);
    L.ftbl = at<int2>(w, lo.o_ftbl[l]);
    L.ttbl = at<int2>(w, lo.o_ttbl[l]);
    L.reps_d = at<int32_t>(w, lo.o_reps[l]);
    L.sel_d = at<int32_t>(w, lo.o_sel[l]);
    L.nc3_d = at<int32_t>(w, lo.o_nc3[l]);
    L.overflow = at<int32_t>(w, lo.o_overflow[l]);
    L.ltbl = at<int2>(w, lo.o_ltbl[l]);
    L.lftbl = at<int2>(w, lo.o_lftbl[l]);
    L.lsel_d = at<int32_t>(w, lo.o_lsel[l]);
  }
  c->ln[0].s = c->stream;   // lane 1's stream is created by the first live round
  c->dg_d = at<double>(w, lo.o_dg);
  c->red = at<double>(w, lo.o_red);
  c->dlx = at<double>(w, lo.o_dl[0]); c->dly = at<double>(w, lo.o_dl[1]); c->dlz = at<double>(w, lo.o_dl[2]);
  c->tdlx = at<double>(w, lo.o_tdl[0]); c->tdly = at<double>(w, lo.o_tdl[1]); c->tdlz = at<double>(w, lo.o_tdl[2]);
  c->alt4 = at<double4>(w, lo.o_alt4);
  c->talt4 = at<double4>(w, lo.o_talt4);
  c->evals = at<unsigned long long>(w, lo.o_evals);
  c->xref4 = at<double4>(w, lo.o_xref4);
  c->zbuf = at<uint16_t>(w, lo.o_zbuf);
  c->lpart = at<double>(w, lo.o_lpart);
  c->mlp = at<MlpDev>(w, lo.o_mlp);
  c->mlpw = at<float>(w, lo.o_mlpw);
  c->tord = at<int32_t>(w, lo.o_tord);
  c->lin = at<LinState>(w, lo.o_lin);

  const size_t tcap = table_cap(std::max(lo.blocks, lo.tiles));
  bool pinned = hipHostMalloc((void**)&c->h_state, sizeof(State) * n_rep, hipHostMallocDefault) == hipSuccess &&
                hipHostMalloc((void**)&c->h_dg, sizeof(double) * 4 * n_rep, hipHostMallocDefault) == hipSuccess;
  for (Lane& L : c->ln)
    pinned = pinned &&
             hipHostMalloc((void**)&L.h_tbl, sizeof(int2) * tcap, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_ftbl, sizeof(int2) * tcap, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_tbl2, sizeof(int2) * tcap, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_ttbl, sizeof(int2) * tcap, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_ltbl, sizeof(int2) * tcap, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_lftbl, sizeof(int2) * tcap, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_reps, sizeof(int32_t) * n_rep, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_sel, sizeof(int32_t) * n_rep, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_lsel, sizeof(int32_t) * n_rep, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_nc3, sizeof(int32_t) * kGridInts * n_rep, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&L.h_over, sizeof(int32_t), hipHostMallocDefault) == hipSuccess;
  if (!pinned) {
    free_pinned(c);
    delete c;
    return fail(AQS_EHIP, "hipHostMalloc of the host staging buffers failed");
  }
  for (Lane& L : c->ln) *L.h_over = 0;
  std::memset(c->h_state, 0, sizeof(State) * n_rep);
  for (int r = 0; r < n_rep; ++r) {
    c->h_state[r].phase = PH_IDLE;
    c->h_state[r].snap_dst = -1;
    reset_minimizer(c, c->h_state[r]);
  }
  c->loaded.assign(n_rep, 0);
  c->dirty.assign(n_rep, 1);
  c->tiles_now.assign(n_rep, 0);
  hipStream_t s = c->stream;
  if (hipMemsetAsync(c->ws, 0, lo.total, s) != hipSuccess ||
      hipMemcpyAsync(c->d_geom, lo.geom.data(), sizeof(Geom) * n_rep, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(c->d_state, c->h_state, sizeof(State) * n_rep, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    free_pinned(c);
    delete c;
    return fail(AQS_EHIP, "initialising the workspace failed");
  }
  *out = c;
  return AQS_OK;
}

aqs_status aqs_destroy(aqs_ctx* c) {
  if (!c) return AQS_OK;
  (void)hipStreamSynchronize(c->stream);
  if (c->ln[1].s) {
    (void)hipStreamSynchronize(c->ln[1].s);
    (void)hipStreamDestroy(c->ln[1].s);
  }
  for (Lane& L : c->ln) drop_graph(L);
  for (Lane& L : c->ln)
    for (hipEvent_t e : L.ev) (void)hipEventDestroy(e);
  free_pinned(c);
  delete c;
  return AQS_OK;
}

aqs_status aqs_set_replica(aqs_ctx* c, int32_t rep, const uint8_t* types, const double* pos,
                           int64_t strain_index) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (rep < 0 || rep >= c->n_rep) return fail(AQS_EINVAL, "slot %d out of range", rep);
  if (!types || !pos) return fail(AQS_EINVAL, "null types or positions");
  const Geom& g = c->lo.geom[rep];
  const int d = c->dim;
  std::vector<double4> p(g.n);
  std::vector<int32_t> ids(g.n);
  for (int i = 0; i < g.n; ++i) {
    if (types[i] > 1) return fail(AQS_EINVAL, "atom %d: type %d not in {0, 1}", i, (int)types[i]);
    p[i] = make_double4(pos[i * d], pos[i * d + 1], d == 3 ? pos[i * d + 2] : 0.0, (double)types[i]);
    ids[i] = i;
  }
  aqs_status st = pull_state(c);
  if (st) return st;
  HIPCHK(hipMemcpyAsync(c->pos4 + g.atom_off, p.data(), sizeof(double4) * g.n,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->id + g.atom_off, ids.data(), sizeof(int32_t) * g.n,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->inv + g.atom_off, ids.data(), sizeof(int32_t) * g.n,
                        hipMemcpyHostToDevice, c->stream));
  State& s = c->h_state[rep];
  s.k = strain_index;
  s.phase = PH_IDLE;
  s.E = 0.0;
  s.fmax = 0.0;
  s.status = 0;
  reset_minimizer(c, s);
  st = push_state(c);
  if (st) return st;
  c->loaded[rep] = 1;
  c->dirty[rep] = 1;
  return AQS_OK;
}

aqs_status aqs_set_positions(aqs_ctx* c, int32_t rep, const double* pos) {
  aqs_status st = check_slot(c, rep);
  if (st) return st;
  if (!pos) return fail(AQS_EINVAL, "null positions");
  const Geom& g = c->lo.geom[rep];
  const int d = c->dim;
  // keep each atom's type, put the atoms back in atom-id order
  std::vector<double4> p(g.n), q(g.n);
  std::vector<int32_t> idv(g.n), ids(g.n);
  HIPCHK(hipMemcpyAsync(p.data(), c->pos4 + g.atom_off, sizeof(double4) * g.n,
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(idv.data(), c->id + g.atom_off, sizeof(int32_t) * g.n,
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int s = 0; s < g.n; ++s) q[idv[s]].w = p[s].w;
  for (int i = 0; i < g.n; ++i) {
    q[i].x = pos[i * d];
    q[i].y = pos[i * d + 1];
    q[i].z = d == 3 ? pos[i * d + 2] : 0.0;
    ids[i] = i;
  }
  HIPCHK(hipMemcpyAsync(c->pos4 + g.atom_off, q.data(), sizeof(double4) * g.n,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->id + g.atom_off, ids.data(), sizeof(int32_t) * g.n,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->inv + g.atom_off, ids.data(), sizeof(int32_t) * g.n,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->dirty[rep] = 1;
  return AQS_OK;
}

aqs_status aqs_get_positions(aqs_ctx* c, int32_t rep, double* pos) {
  aqs_status st = check_slot(c, rep);
  if (st) return st;
  if (!pos) return fail(AQS_EINVAL, "null output");
  const Geom& g = c->lo.geom[rep];
  const int d = c->dim;
  std::vector<double4> p(g.n);
  std::vector<int32_t> idv(g.n);
  HIPCHK(hipMemcpyAsync(p.data(), c->pos4 + g.atom_off, sizeof(double4) * g.n,
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(idv.data(), c->id + g.atom_off, sizeof(int32_t) * g.n,
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int s = 0; s < g.n; ++s) {
    const int i = idv[s];
    pos[i * d] = p[s].x;
    pos[i * d + 1] = p[s].y;
    if (d == 3) pos[i * d + 2] = p[s].z;
  }
  return AQS_OK;
}

aqs_status aqs_get_strain_index(aqs_ctx* c, int32_t rep, int64_t* k) {
  aqs_status st = check_slot(c, rep);
  if (st) return st;
  st = pull_state(c);
  if (st) return st;
  if (k) *k = c->h_state[rep].k;
  return AQS_OK;
}

aqs_status aqs_get_box(aqs_ctx* c, int32_t rep, double* H) {
  if (!c || !H) return fail(AQS_EINVAL, "null argument");
  if (rep < 0 || rep >= c->n_rep) return fail(AQS_EINVAL, "slot %d out of range [0, %d)", rep, c->n_rep);
  aqs_status st = pull_state(c);
  if (st) return st;
  const Box b = box_of(c, rep, c->h_state[rep].k);
  const int d = c->dim;
  for (int x = 0; x < d * d; ++x) H[x] = 0.0;
  H[0] = b.h00;
  H[1] = b.h01;
  H[d] = b.h10;
  H[d + 1] = b.h11;
  if (d == 3) H[8] = b.h22;
  return AQS_OK;
}

aqs_status aqs_copy_replica(aqs_ctx* c, int32_t src, int32_t dst) {
  aqs_status st = check_slot(c, src);
  if (st) return st;
  if (dst < 0 || dst >= c->n_rep) return fail(AQS_EINVAL, "slot %d out of range", dst);
  if (dst == src) return AQS_OK;
  if (c->lo.geom[src].n != c->lo.geom[dst].n)
    return fail(AQS_EINVAL, "slots %d and %d differ in atom count", src, dst);
  if (c->lo.geom[src].dgamma_y != c->lo.geom[dst].dgamma_y ||
      c->lo.geom[src].dgamma != c->lo.geom[dst].dgamma)
    return fail(AQS_EINVAL, "slots %d and %d differ in their deformation (shear mode or dgamma)", src, dst);
  st = pull_state(c);
  if (st) return st;
  launch_copy_slot(c->d_geom, src, dst, c->lo.geom[src].n, c->pos4, c->id, c->inv, c->stream);
  HIPCHK(hipGetLastError());
  State& d = c->h_state[dst];
  const State& s = c->h_state[src];
  d.k = s.k;
  d.E = s.E;
  d.fmax = s.fmax;
  d.sxy = s.sxy;
  d.status = s.status;
  d.phase = PH_IDLE;
  reset_minimizer(c, d);
  st = push_state(c);
  if (st) return st;
  c->loaded[dst] = 1;
  c->dirty[dst] = 1;
  return AQS_OK;
}

aqs_status aqs_affine_shear(aqs_ctx* c, int32_t n_sel, const int32_t* rep, const int64_t* dk) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (n_sel <= 0) return AQS_OK;
  if (!rep || !dk) return fail(AQS_EINVAL, "null selection");
  std::vector<int32_t> sel(rep, rep + n_sel);
  // a slot listed twice would get two blocks per atom block in the launch
  // table, racing on x += dg y, while its strain index took both dk
  std::vector<char> seen(c->n_rep, 0);
  for (int r : sel) {
    aqs_status st = check_slot(c, r);
    if (st) return st;
    if (seen[r]) return fail(AQS_EINVAL, "slot %d selected twice", r);
    seen[r] = 1;
  }
  aqs_status st = pull_state(c);
  if (st) return st;
  for (int i = 0; i < n_sel; ++i) {
    const Geom& g = c->lo.geom[sel[i]];
    if (g.dgamma_y != 0.0 && (dk[i] < 0 || c->h_state[sel[i]].k + dk[i] < 0))
      return fail(AQS_EINVAL, "slot %d: a pure shear is only applied forward (dk %lld)", sel[i],
                  (long long)dk[i]);
  }
  // per slot the 2x2 map of (x, y): simple shear F^dk = [[1, dk dgamma], [0, 1]]
  // with dk dgamma in one multiplication (level I, Eq. 18); the pure shear's
  // F^dk by the same square-and-multiply as its box
  std::vector<double> dg(4 * (size_t)c->n_rep, 0.0);
  for (int i = 0; i < n_sel; ++i) {
    const Geom& g = c->lo.geom[sel[i]];
    double* M = &dg[4 * (size_t)sel[i]];
    if (g.dgamma_y == 0.0) {
      M[0] = 1.0;
      M[1] = (double)dk[i] * g.dgamma;
      M[3] = 1.0;
    } else {
      deformation_power(g.dgamma, g.dgamma_y, dk[i], M);
    }
    c->h_state[sel[i]].k += dk[i];
  }
  Lane& L = c->ln[0];
  std::vector<int2> tbl = make_table(c, sel, L.xcd_mask);
  std::copy(tbl.begin(), tbl.end(), L.h_tbl2);
  std::copy(dg.begin(), dg.end(), c->h_dg);
  HIPCHK(hipMemcpyAsync(L.tbl2, L.h_tbl2, sizeof(int2) * tbl.size(), hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipMemcpyAsync(c->dg_d, c->h_dg, sizeof(double) * 4 * c->n_rep, hipMemcpyHostToDevice,
                        c->stream));
  launch_affine(L.tbl2, (int32_t)tbl.size(), c->d_geom, c->pos4, c->dg_d, c->stream);
  HIPCHK(hipGetLastError());
  return push_state(c);
}

aqs_status aqs_minimize_batch(aqs_ctx* c, int32_t n_sel, const int32_t* rep, int32_t start_mode,
                              const int32_t* n_steps, const int32_t* snap_dst,
                              aqs_step_record* records) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (n_sel <= 0) return AQS_OK;
  if (!rep) return fail(AQS_EINVAL, "null selection");
  std::vector<int32_t> sel(rep, rep + n_sel);
  aqs_status st = start_chains(c, sel, start_mode, n_steps, snap_dst);
  if (st) return st;
  Lane& L = c->ln[0];
  st = set_table(c, L, sel);
  if (st) return st;
  launch_reset_iter(L.tbl, L.cur_nblk, c->d_geom, c->vx, c->vy, c->vz, c->upart, c->dim, L.s);
  HIPCHK(hipGetLastError());
  for (;;) {
    st = lane_launch(c, L, start_mode, true);
    if (st) return st;
    int active = 0;
    st = lane_poll(c, L, true, active);
    if (st) return st;
    if (!active) break;
  }
  return finish_chains(c, sel, n_steps, snap_dst, std::vector<char>(sel.size(), 0), records);
}


aqs_status aqs_run_round(aqs_ctx* c, int32_t P, const int32_t* chain, const int32_t* snap,
                         const int32_t* n_steps, int32_t start_mode, double delta_eq,
                         int32_t live, aqs_step_record* records, aqs_check* checks) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (P <= 0 || !chain || !n_steps || !checks) return fail(AQS_EINVAL, "bad round arguments");
  if (P > 1 && !snap) return fail(AQS_EINVAL, "a round of several chains needs snapshot slots");
  for (int i = 1; i < P; ++i)
    if (snap[i] < 0) return fail(AQS_EINVAL, "chain %d has no snapshot slot", i);
  std::vector<int32_t> sel(chain, chain + P), snp(P, -1);
  for (int i = 1; i < P; ++i) snp[i] = snap[i];
  for (int i = 0; i < P; ++i) checks[i] = aqs_check{0, 0, 0.0, 0.0};
  aqs_status st = start_chains(c, sel, start_mode, n_steps, snp.data());
  if (st) return st;
  std::vector<char> cancelled(P, 0);
  Lane& B = c->ln[0];
  if (live < 0 || live > 2) return fail(AQS_EINVAL, "live must be 0, 1 or 2 (got %d)", live);
  const bool abandon = (live == 2);
  if (!live || P == 1) {
    // all chains to completion on the context stream, then the checks in order
    st = set_table(c, B, sel);
    if (st) return st;
    launch_reset_iter(B.tbl, B.cur_nblk, c->d_geom, c->vx, c->vy, c->vz, c->upart, c->dim, B.s);
    HIPCHK(hipGetLastError());
    for (;;) {
      st = lane_launch(c, B, start_mode, true);
      if (st) return st;
      int active = 0;
      st = lane_poll(c, B, true, active);
      if (st) return st;
      if (!active) break;
    }
    for (int i = 1; i < P; ++i) {
      st = compare_slots(c, B, chain[i - 1], snp[i], delta_eq, &checks[i]);
      if (st) return st;
      if (!checks[i].equal) break;
    }
    return finish_chains(c, sel, n_steps, snp.data(), cancelled, records);
  }
  // live: the critical chain (the first one whose end a pending check needs)
  // runs alone on lane 1, the others on lane 0; each check is taken as soon
  // as both of its configurations exist; a failed check stops the chains
  // after it.
  Lane& C = c->ln[1];
  if (!C.s) HIPCHK(hipStreamCreateWithFlags(&C.s, hipStreamNonBlocking));
  c->live = true;
  struct LiveOff {
    aqs_ctx* c;
    ~LiveOff() {
      c->live = false;
      for (Lane& L : c->ln) L.xcd_mask = kAllXcds;
    }
  } live_off{c};
  if (c->tn.live_xcds > 0) {
    // the critical chain's blocks on the last live_xcds XCDs, the batch's on
    // the others: each keeps its own compute units and L2
    C.xcd_mask = kAllXcds & ~((1u << (kXcds - c->tn.live_xcds)) - 1u);
    B.xcd_mask = kAllXcds & ~C.xcd_mask;
  }
  st = set_table(c, C, std::vector<int32_t>{chain[0]});
  if (st) return st;
  st = set_table(c, B, std::vector<int32_t>(chain + 1, chain + P));
  if (st) return st;
  for (Lane* L : {&C, &B}) {
    launch_reset_iter(L->tbl, L->cur_nblk, c->d_geom, c->vx, c->vy, c->vz, c->upart, c->dim, L->s);
    HIPCHK(hipGetLastError());
  }
  int next = 1;   // next check
  // duty cycle of the batch while a critical chain runs (live_duty D > 1):
  // after a block of the batch that took T, the batch waits (D - 1) T, so the
  // critical chain runs alone that long
  using clk = std::chrono::steady_clock;
  clk::time_point b_start = clk::now(), b_idle_until = b_start;
  for (;;) {
    for (Lane* L : {&C, &B})
      if (!L->in_flight && lane_active(c, *L)) {
        if (L == &B && c->tn.live_duty > 1 && lane_active(c, C) && clk::now() < b_idle_until)
          continue;
        st = lane_launch(c, *L, start_mode, true);
        if (st) return st;
        if (L == &B) b_start = clk::now();
      }
    if (!C.in_flight && !B.in_flight) {
      if (!lane_active(c, B) || !lane_active(c, C)) break;
      continue;   // the batch waits out its idle time while the critical chain is between blocks
    }
    // wait for either lane's block: a blocking wait when one lane is in flight,
    // else both polled without sleeping (a sleep's wake-up latency would idle
    // the critical chain between its blocks)
    Lane* done = nullptr;
    if (C.in_flight != B.in_flight) {
      done = C.in_flight ? &C : &B;
      HIPCHK(hipStreamSynchronize(done->s));
    }
    while (!done) {
      for (Lane* L : {&C, &B}) {
        if (!L->in_flight) continue;
        const hipError_t q = hipStreamQuery(L->s);
        if (q == hipSuccess) {
          done = L;
          break;
        }
        if (q != hipErrorNotReady) return fail(AQS_EHIP, "hipStreamQuery: %s", hipGetErrorString(q));
      }
      if (!done) std::this_thread::yield();
    }
    int active = 0;
    st = lane_poll(c, *done, false, active);
    if (st) return st;
    if (done == &B && c->tn.live_duty > 1) {
      const clk::time_point now = clk::now();
      b_idle_until = now + (now - b_start) * (c->tn.live_duty - 1);
    }
    // a plastic event in the critical chain, still running, predicts that
    // the check on its end fails: the chains after it are stopped now (once
    // the chain is done, the check itself is taken below)
    if (abandon && next < P && done == &C && c->h_state[chain[next - 1]].drops > 0 &&
        c->h_state[chain[next - 1]].phase != PH_DONE) {
      if (B.in_flight) {
        HIPCHK(hipStreamSynchronize(B.s));
        st = lane_poll(c, B, false, active);
        if (st) return st;
      }
      std::vector<int32_t> stop;
      for (int j = next; j < P; ++j)
        if (c->h_state[chain[j]].phase != PH_DONE) {
          c->h_state[chain[j]].phase = PH_DONE;
          cancelled[j] = 1;
          stop.push_back(chain[j]);
        }
      st = push_slots(c, B, stop);
      if (st) return st;
      checks[next] = aqs_check{2, 0, 0.0, 0.0};
      next = P;
      st = set_table(c, B, std::vector<int32_t>{});
      if (st) return st;
    }
    // checks whose configurations are ready, in order
    while (next < P) {
      const int i = next;
      if (c->h_state[chain[i - 1]].phase != PH_DONE) break;         // end of chain i-1
      const State& si = c->h_state[chain[i]];
      if (!(si.step >= 1 || si.phase == PH_DONE)) break;             // first IS of chain i
      st = compare_slots(c, C, chain[i - 1], snp[i], delta_eq, &checks[i]);
      if (st) return st;
      // lane 0 idle before its selection changes
      if (B.in_flight) {
        HIPCHK(hipStreamSynchronize(B.s));
        st = lane_poll(c, B, false, active);
        if (st) return st;
      }
      ++next;
      std::vector<int32_t> rest;
      if (checks[i].equal) {
        // chain i becomes the critical chain
        for (int r : B.cur_sel)
          if (r != chain[i]) rest.push_back(r);
        st = set_table(c, C, std::vector<int32_t>{chain[i]});
        if (st) return st;
      } else {
        // chains i .. P-1 are rejected by Algorithm 1: stop them
        std::vector<int32_t> stop;
        for (int j = i; j < P; ++j)
          if (c->h_state[chain[j]].phase != PH_DONE) {
            c->h_state[chain[j]].phase = PH_DONE;
            cancelled[j] = 1;
            stop.push_back(chain[j]);
          }
        st = push_slots(c, B, stop);
        if (st) return st;
        next = P;
      }
      st = set_table(c, B, rest);
      if (st) return st;
    }
  }
  HIPCHK(hipStreamSynchronize(C.s));
  HIPCHK(hipStreamSynchronize(B.s));
  return finish_chains(c, sel, n_steps, snp.data(), cancelled, records);
}

aqs_status aqs_compare_configs(aqs_ctx* c, int32_t ra, int32_t rb, double delta_eq,
                               int32_t* equal, double* max_disp, double* de_per_atom) {
  aqs_status st = check_slot(c, ra);
  if (st) return st;
  st = check_slot(c, rb);
  if (st) return st;
  const Geom& g = c->lo.geom[ra];
  if (g.n != c->lo.geom[rb].n) return fail(AQS_EINVAL, "slots differ in atom count");
  if (g.dgamma_y != c->lo.geom[rb].dgamma_y || g.dgamma != c->lo.geom[rb].dgamma)
    return fail(AQS_EINVAL, "slots differ in their deformation");
  st = pull_state(c);
  if (st) return st;
  if (c->h_state[ra].k != c->h_state[rb].k)
    return fail(AQS_EINVAL, "slots %d and %d are at different strain indices (%lld vs %lld)", ra,
                rb, (long long)c->h_state[ra].k, (long long)c->h_state[rb].k);
  const int nb = (g.n + kBlock - 1) / kBlock;
  launch_compare(c->d_geom, ra, rb, g.n, c->pos4, c->inv, box_of(c, ra, c->h_state[ra].k), c->dim,
                 c->red, c->stream);
  HIPCHK(hipGetLastError());
  std::vector<double> part(nb);
  HIPCHK(hipMemcpyAsync(part.data(), c->red, sizeof(double) * nb, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double m = 0.0;
  for (double v : part) m = std::max(m, v);
  if (max_disp) *max_disp = m;
  if (de_per_atom) *de_per_atom = (c->h_state[ra].E - c->h_state[rb].E) / (double)g.n;
  if (equal) *equal = (m < delta_eq) ? 1 : 0;
  return AQS_OK;
}

aqs_status aqs_stress(aqs_ctx* c, int32_t rep, double* sigma, double* energy) {
  aqs_status st = check_slot(c, rep);
  if (st) return st;
  st = pull_state(c);
  if (st) return st;
  std::vector<int32_t> sel(1, rep);
  st = rebuild(c, c->ln[0], sel, false, 1);  // global-index entries for the virial kernel
  if (st) return st;
  const Geom& g = c->lo.geom[rep];
  IterArgs a = iter_args(c, c->ln[0]);
  const Box bx = box_of(c, rep, c->h_state[rep].k);
  launch_virial(a, rep, g.nblocks, c->dim, bx, c->red, c->stream);
  HIPCHK(hipGetLastError());
  std::vector<double> part((size_t)g.nblocks * 10);
  HIPCHK(hipMemcpyAsync(part.data(), c->red, sizeof(double) * part.size(), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double tot[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < g.nblocks; ++b)
    for (int k = 0; k < 10; ++k) tot[k] += part[(size_t)b * 10 + k];
  // simple shear keeps V = Lx Ly Lz; the pure shear of Eq. (17) scales the (x, y) area
  const double vol = (bx.h10 == 0.0) ? g.L[0] * g.L[1] * g.L[2]
                                     : std::fabs(bx.h00 * bx.h11 - bx.h01 * bx.h10) * bx.h22;
  const int d = c->dim;
  if (sigma)
    for (int x = 0; x < d; ++x)
      for (int y = 0; y < d; ++y) sigma[x * d + y] = tot[1 + 3 * x + y] / vol;
  if (energy) *energy = tot[0];
  return AQS_OK;
}

aqs_status aqs_energy_forces(aqs_ctx* c, int32_t rep, double* energy, double* forces) {
  aqs_status st = check_slot(c, rep);
  if (st) return st;
  st = pull_state(c);
  if (st) return st;
  std::vector<int32_t> sel(1, rep);
  Lane& L = c->ln[0];
  st = rebuild(c, L, sel);
  if (st) return st;
  c->h_state[rep].phase = PH_EVAL;
  st = push_state(c);
  if (st) return st;
  st = set_table(c, L, sel);
  if (st) return st;
  IterArgs a = iter_args(c, L);
  launch_force(a, L.cur_ntiles, c->dim, c->stream);
  launch_control(a, c->stream);
  HIPCHK(hipGetLastError());
  st = pull_state(c);
  if (st) return st;
  if (c->h_state[rep].phase != PH_DONE)
    return fail(AQS_ESTATE, "force evaluation of slot %d did not complete (phase %d)", rep,
                c->h_state[rep].phase);
  c->h_state[rep].phase = PH_IDLE;
  st = push_state(c);
  if (st) return st;
  if (energy) *energy = c->h_state[rep].E;
  if (forces) {
    const Geom& g = c->lo.geom[rep];
    const int d = c->dim;
    std::vector<double> f[3];
    for (int k = 0; k < d; ++k) f[k].resize(g.n);
    std::vector<int32_t> idv(g.n);
    double* src[3] = {c->fx, c->fy, c->fz};
    for (int k = 0; k < d; ++k)
      HIPCHK(hipMemcpyAsync(f[k].data(), src[k] + g.atom_off, sizeof(double) * g.n,
                            hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(idv.data(), c->id + g.atom_off, sizeof(int32_t) * g.n,
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int s = 0; s < g.n; ++s)
      for (int k = 0; k < d; ++k) forces[idv[s] * d + k] = f[k][s];
  }
  return AQS_OK;
}

aqs_status aqs_set_minimizer(aqs_ctx* c, int32_t minimizer, const aqs_cg_params* cg) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (minimizer == AQS_MIN_FIRE) {
    c->minimizer = kMinFire;
    for (Lane& L : c->ln) drop_graph(L);   // captured launches hold the minimiser's kernels
    return AQS_OK;
  }
  if (minimizer != AQS_MIN_CG) return fail(AQS_EINVAL, "unknown minimizer %d", minimizer);
  if (!cg) return fail(AQS_EINVAL, "AQS_MIN_CG needs its parameters");
  if (!(cg->a_init > 0.0) || !(cg->sigma > 0.0 && cg->sigma < 1.0) || !(cg->grow > 1.1) ||
      !(cg->dmax > 0.0) || !(cg->ftol > 0.0) || cg->ls_max < 1 || cg->n_fail_max < 0 ||
      cg->max_iter < 1)
    return fail(AQS_EINVAL, "conjugate-gradient parameters out of range");
  CgParams p{};
  p.a_init = cg->a_init;
  p.sigma = cg->sigma;
  p.grow = cg->grow;
  p.dmax = cg->dmax;
  p.ftol = cg->ftol;
  p.ls_max = cg->ls_max;
  p.n_fail_max = cg->n_fail_max;
  p.max_iter = cg->max_iter;
  c->cg = p;
  c->minimizer = kMinCG;
  for (Lane& L : c->ln) drop_graph(L);   // captured launches hold the parameters
  return AQS_OK;
}

aqs_status aqs_set_live_batch_blocks(aqs_ctx* c, int32_t blocks) {
  if (!c) return fail(AQS_EINVAL, "null context");
  c->tn.live_blocks = blocks < 0 ? 0 : (blocks == 0 ? 3 : std::min(blocks, 4));
  c->live_pad = -1;   // recomputed for the new limit at the next live launch
  return AQS_OK;
}

aqs_status aqs_set_live_xcds(aqs_ctx* c, int32_t xcds) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (xcds < 0 || xcds >= kXcds) return fail(AQS_EINVAL, "live_xcds %d outside [0, %d]", xcds, kXcds - 1);
  c->tn.live_xcds = xcds;
  return AQS_OK;
}

aqs_status aqs_set_dgamma(aqs_ctx* c, int32_t n_sel, const int32_t* rep, const double* dgamma) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (n_sel <= 0) return AQS_OK;
  if (!rep || !dgamma) return fail(AQS_EINVAL, "null selection");
  aqs_status st = pull_state(c);
  if (st) return st;
  std::vector<int64_t> knew(n_sel, 0), kbnew(n_sel, 0);
  for (int i = 0; i < n_sel; ++i) {
    const int r = rep[i];
    if (r < 0 || r >= c->n_rep) return fail(AQS_EINVAL, "slot %d out of range [0, %d)", r, c->n_rep);
    const Geom& g = c->lo.geom[r];
    const double d = dgamma[i];
    if (!std::isfinite(d) || d == 0.0) return fail(AQS_EINVAL, "slot %d: dgamma %g", r, d);
    if (g.dgamma_y != 0.0) return fail(AQS_EINVAL, "slot %d is pure-sheared: its box depends on dgamma", r);
    const State& s = c->h_state[r];
    if (s.phase != PH_IDLE && s.phase != PH_DONE)
      return fail(AQS_ESTATE, "slot %d is running (phase %d)", r, s.phase);
    // the strain k dgamma is kept exactly: the new index is an integer and
    // forms the same strain (and so the same box) in one product
    for (int w = 0; w < 2; ++w) {
      const int64_t k = w == 0 ? s.k : s.k_build;
      const double kd = std::nearbyint((double)k * g.dgamma / d);
      const int64_t kn = (int64_t)kd;
      if (strain_of(kn, d) != strain_of(k, g.dgamma)) {
        if (w == 1) {   // the list is rebuilt at the next call anyway
          kbnew[i] = kn;
          continue;
        }
        return fail(AQS_EINVAL, "slot %d: strain %g is not a multiple of dgamma %g", r,
                    strain_of(k, g.dgamma), d);
      }
      (w == 0 ? knew : kbnew)[i] = kn;
    }
  }
  for (int i = 0; i < n_sel; ++i) {
    const int r = rep[i];
    c->lo.geom[r].dgamma = dgamma[i];
    c->h_state[r].k = knew[i];
    c->h_state[r].k_build = kbnew[i];
    c->dirty[r] = 1;
  }
  st = push_state(c);
  if (st) return st;
  HIPCHK(hipMemcpyAsync(c->d_geom, c->lo.geom.data(), sizeof(Geom) * c->n_rep, hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return AQS_OK;
}

aqs_status aqs_set_linear_start(aqs_ctx* c, int32_t max_cg, double tol, double probe) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (max_cg < 1 || max_cg > 100000) return fail(AQS_EINVAL, "max_cg %d outside [1, 100000]", max_cg);
  if (!(tol > 0.0 && tol < 1.0)) return fail(AQS_EINVAL, "tol %g outside (0, 1)", tol);
  if (!(probe > 0.0 && probe < 0.1)) return fail(AQS_EINVAL, "probe %g outside (0, 0.1)", probe);
  c->tn.lin_max_cg = max_cg;
  c->tn.lin_tol = tol;
  c->tn.lin_probe = probe;
  return AQS_OK;
}

aqs_status aqs_set_live_duty(aqs_ctx* c, int32_t duty) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (duty < 1 || duty > 64) return fail(AQS_EINVAL, "live duty %d outside [1, 64]", duty);
  c->tn.live_duty = duty;
  return AQS_OK;
}

aqs_status aqs_set_pure_shear(aqs_ctx* c, int32_t n_sel, const int32_t* rep,
                              const double* dgamma_y) {
  if (!c) return fail(AQS_EINVAL, "null context");
  if (n_sel <= 0) return AQS_OK;
  if (!rep || !dgamma_y) return fail(AQS_EINVAL, "null selection");
  for (int i = 0; i < n_sel; ++i) {
    const int r = rep[i];
    if (r < 0 || r >= c->n_rep) return fail(AQS_EINVAL, "slot %d out of range [0, %d)", r, c->n_rep);
    const double b = dgamma_y[i];
    if (!std::isfinite(b) || !(std::fabs(c->lo.geom[r].dgamma * b) < 1.0))
      return fail(AQS_EINVAL, "slot %d: dgamma_y %g gives a singular deformation", r, b);
  }
  aqs_status st = pull_state(c);
  if (st) return st;
  for (int i = 0; i < n_sel; ++i) {
    const int ph = c->h_state[rep[i]].phase;
    if (ph != PH_IDLE && ph != PH_DONE)
      return fail(AQS_ESTATE, "slot %d is running (phase %d)", rep[i], ph);
    if (dgamma_y[i] != 0.0 && c->h_state[rep[i]].k < 0)
      return fail(AQS_EINVAL, "slot %d: pure shear needs a strain index >= 0", rep[i]);
  }
  for (int i = 0; i < n_sel; ++i) {
    c->lo.geom[rep[i]].dgamma_y = dgamma_y[i];
    c->dirty[rep[i]] = 1;
  }
  HIPCHK(hipMemcpyAsync(c->d_geom, c->lo.geom.data(), sizeof(Geom) * c->n_rep, hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return AQS_OK;
}

aqs_status aqs_set_profiling(aqs_ctx* c, int32_t every_nth_block) {
  if (!c) return fail(AQS_EINVAL, "null context");
  c->prof_every = every_nth_block > 0 ? every_nth_block : 0;
  c->block_count = 0;
  return AQS_OK;
}

aqs_status aqs_get_counters(aqs_ctx* c, aqs_counters* out, int32_t reset) {
  if (!c) return fail(AQS_EINVAL, "null context");
  unsigned long long ev[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(ev, c->evals, sizeof ev, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->cnt.atom_evals = (int64_t)ev[0] + c->lin_evals;
  c->cnt.timed_atom_evals = (int64_t)ev[1];
  if (out) *out = c->cnt;
  if (reset) {
    c->cnt = aqs_counters{};
    c->lin_evals = 0;
    HIPCHK(hipMemsetAsync(c->evals, 0, sizeof ev, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return AQS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned start

namespace {

// Device buffers of one training or gradient call.
struct TrainPtrs {
  uint16_t* z = nullptr;
  float *t = nullptr, *part = nullptr, *master = nullptr, *m = nullptr, *v = nullptr,
        *grad = nullptr;
  double *stats = nullptr, *stat_part = nullptr, *loss = nullptr;
  int32_t* order = nullptr;
  uint8_t* keep = nullptr;
  MlpDev* mlp = nullptr;
};

// ... allocated by the call itself (freed by the destructor).
struct TrainBufs : TrainPtrs {
  ~TrainBufs() {
    void* ps[] = {z, t, stats, part, master, m, v, grad, stat_part, loss, order, keep, mlp};
    for (void* p : ps)
      if (p) (void)hipFree(p);
  }
};

aqs_status train_alloc(TrainBufs& b, int64_t n, int32_t blocks, int32_t epochs, bool adam) {
  auto al = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 256)); };
  if (al((void**)&b.z, sizeof(uint16_t) * kFeat * n) != hipSuccess ||
      al((void**)&b.t, sizeof(float) * 4 * n) != hipSuccess ||
      al((void**)&b.stats, sizeof(double) * 2 * 68) != hipSuccess ||
      al((void**)&b.stat_part, sizeof(double) * 65 * 256) != hipSuccess ||
      al((void**)&b.keep, sizeof(uint8_t) * n) != hipSuccess ||
      al((void**)&b.part, sizeof(float) * (size_t)(kNumParams + 1) * blocks) != hipSuccess ||
      al((void**)&b.master, sizeof(float) * kNumParams) != hipSuccess ||
      al((void**)&b.loss, sizeof(double) * std::max(epochs, 1)) != hipSuccess ||
      al((void**)&b.mlp, sizeof(MlpDev)) != hipSuccess)
    return fail(AQS_EHIP, "device allocation for the network failed");
  if (adam && (al((void**)&b.m, sizeof(float) * kNumParams) != hipSuccess ||
               al((void**)&b.v, sizeof(float) * kNumParams) != hipSuccess))
    return fail(AQS_EHIP, "device allocation for the optimiser failed");
  if (!adam && al((void**)&b.grad, sizeof(float) * kNumParams) != hipSuccess)
    return fail(AQS_EHIP, "device allocation for the gradient failed");
  return AQS_OK;
}

// Network parameters (flat FP32, the order of aqs_mlp) of a model.
const float* params_of(const aqs_mlp* m) { return &m->w1[0]; }
float* params_of(aqs_mlp* m) { return &m->w1[0]; }

aqs_status upload_mlp(hipStream_t s, const aqs_mlp* m, float* master, MlpDev* dev, bool stats) {
  HIPCHK(hipMemcpyAsync(master, params_of(m), sizeof(float) * kNumParams, hipMemcpyHostToDevice, s));
  const int32_t dim = m->dim;
  HIPCHK(hipMemcpyAsync(&dev->dim, &dim, sizeof dim, hipMemcpyHostToDevice, s));
  if (stats) {
    float tm[4] = {0, 0, 0, 0}, ts[4] = {1, 1, 1, 1};
    for (int k = 0; k < dim; ++k) {
      tm[k] = m->tgt_mean[k];
      ts[k] = m->tgt_std[k];
    }
    HIPCHK(hipMemcpyAsync(dev->fmean, m->feat_mean, sizeof(float) * kFeat, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dev->fstd, m->feat_std, sizeof(float) * kFeat, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dev->tmean, tm, sizeof tm, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dev->tstd, ts, sizeof ts, hipMemcpyHostToDevice, s));
  }
  launch_mlp_sync(master, dev, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return AQS_OK;
}

aqs_status check_mlp(const aqs_mlp* m) {
  if (!m) return fail(AQS_EINVAL, "null network");
  if (m->dim != 2 && m->dim != 3) return fail(AQS_EINVAL, "network dim must be 2 or 3");
  return AQS_OK;
}

// Slot rep alone as the current table, cells and lists rebuilt.
aqs_status prepare_single(aqs_ctx* c, int32_t rep) {
  aqs_status st = check_slot(c, rep);
  if (st) return st;
  st = pull_state(c);
  if (st) return st;
  std::vector<int32_t> sel{rep};
  st = rebuild(c, c->ln[0], sel);
  if (st) return st;
  return set_table(c, c->ln[0], sel);
}

}  // namespace

extern "C" {

aqs_status aqs_learned_load(aqs_ctx* c, const aqs_mlp* m) {
  if (!c) return fail(AQS_EINVAL, "null context");
  aqs_status st = check_mlp(m);
  if (st) return st;
  if (m->dim != c->dim) return fail(AQS_EINVAL, "network has %d outputs, context dim %d", m->dim, c->dim);
  for (int f = 0; f < kFeat; ++f)
    if (!(m->feat_std[f] > 0.0f)) return fail(AQS_EINVAL, "feature std %d not positive", f);
  for (int k = 0; k < m->dim; ++k)
    if (!(m->tgt_std[k] > 0.0f)) return fail(AQS_EINVAL, "target std %d not positive", k);
  st = upload_mlp(c->stream, m, c->mlpw, c->mlp, true);
  if (st) return st;
  c->mlp_dim = m->dim;
  return AQS_OK;
}

aqs_status aqs_learned_features(aqs_ctx* c, int32_t rep, float* feat) {
  if (!c || !feat) return fail(AQS_EINVAL, "null argument");
  aqs_status st = prepare_single(c, rep);
  if (st) return st;
  launch_ldesc(learn_args(c, c->ln[0], 1, feat), c->ln[0].cur_ntiles, c->dim, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return AQS_OK;
}

aqs_status aqs_learned_predict(aqs_ctx* c, int32_t rep, float* u_hat) {
  if (!c || !u_hat) return fail(AQS_EINVAL, "null argument");
  if (c->mlp_dim != c->dim) return fail(AQS_ESTATE, "no network loaded");
  aqs_status st = prepare_single(c, rep);
  if (st) return st;
  launch_ldesc(learn_args(c, c->ln[0], 2), c->ln[0].cur_ntiles, c->dim, c->stream);
  launch_lmlp(learn_args(c, c->ln[0], 1, u_hat), c->ln[0].cur_nblk, c->dim, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return AQS_OK;
}

aqs_status aqs_learned_targets(aqs_ctx* c, int32_t rep_prev, int32_t rep_next, float* target) {
  if (!c || !target) return fail(AQS_EINVAL, "null argument");
  aqs_status st = check_slot(c, rep_prev);
  if (st) return st;
  st = check_slot(c, rep_next);
  if (st) return st;
  const Geom& ga = c->lo.geom[rep_prev];
  const Geom& gb = c->lo.geom[rep_next];
  if (ga.n != gb.n) return fail(AQS_EINVAL, "slots %d and %d differ in size", rep_prev, rep_next);
  if (ga.dgamma != gb.dgamma || ga.dgamma_y != gb.dgamma_y)
    return fail(AQS_EINVAL, "slots differ in their deformation");
  st = pull_state(c);
  if (st) return st;
  const int64_t steps = c->h_state[rep_next].k - c->h_state[rep_prev].k;
  if (steps <= 0 || ga.dgamma == 0.0)
    return fail(AQS_EINVAL, "slot %d is not strained beyond slot %d", rep_next, rep_prev);
  AffineMap f{1.0, (double)steps * ga.dgamma, 0.0, 1.0, (double)steps * ga.dgamma};
  if (ga.dgamma_y != 0.0) {
    double M[4];
    deformation_power(ga.dgamma, ga.dgamma_y, steps, M);
    f = AffineMap{M[0], M[1], M[2], M[3], (double)steps * ga.dgamma};
  }
  launch_ltargets(c->d_geom, rep_prev, rep_next, ga.n, c->pos4, c->inv, c->dim, f,
                  box_of(c, rep_next, c->h_state[rep_next].k), target, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return AQS_OK;
}

}  // extern "C"

namespace {

aqs_status check_train(const aqs_train_params* p, int64_t n, const float* feat,
                       const float* target, const int32_t* order, const aqs_mlp* model) {
  if (!p || !feat || !target || !order) return fail(AQS_EINVAL, "null argument");
  aqs_status st = check_mlp(model);
  if (st) return st;
  if (n <= 0 || p->batch <= 0 || p->epochs <= 0 || n > (int64_t)INT32_MAX)
    return fail(AQS_EINVAL, "bad training sizes");
  if (!(p->huber_delta > 0.0f) || !(p->lr > 0.0f))
    return fail(AQS_EINVAL, "bad training parameters");
  return AQS_OK;
}

// The training of aqs_mlp_train on buffers b, sized for n samples, batches of
// min(p->batch, n) and p->epochs epochs.  Adam's moments and the loss
// accumulators are cleared here by a kernel.
aqs_status train_run(const aqs_train_params* p, int64_t n, const float* feat,
                     const float* target, const int32_t* order, aqs_mlp* model,
                     float* loss_hist, hipStream_t s, const TrainPtrs& b) {
  const int32_t bsz = (int32_t)std::min<int64_t>(p->batch, n);
  launch_zero_words(reinterpret_cast<uint32_t*>(b.m), kNumParams, s);
  launch_zero_words(reinterpret_cast<uint32_t*>(b.v), kNumParams, s);
  launch_zero_words(reinterpret_cast<uint32_t*>(b.loss), 2 * (int64_t)p->epochs, s);
  HIPCHK(hipGetLastError());
  aqs_status st = upload_mlp(s, model, b.master, b.mlp, false);
  if (st) return st;
  TrainArgs a{};
  a.feat = feat;
  a.tgt = target;
  a.n = n;
  a.dim = model->dim;
  a.z = b.z;
  a.t = b.t;
  a.stat_part = b.stat_part;
  a.stats = b.stats;
  a.keep = b.keep;
  a.delta = p->huber_delta;
  a.part = b.part;
  a.master = b.master;
  a.m = b.m;
  a.v = b.v;
  a.mlp = b.mlp;
  a.lr = p->lr;
  a.beta1 = p->beta1;
  a.beta2 = p->beta2;
  a.eps = p->eps;
  launch_train_stats(a, s);
  launch_train_prep(a, s);
  HIPCHK(hipGetLastError());
  int64_t step = 0, batches = 0;
  for (int e = 0; e < p->epochs; ++e) {
    batches = 0;
    for (int64_t b0 = 0; b0 < n; b0 += bsz) {
      a.order = order;
      a.b0 = (int64_t)e * n + b0;
      a.rows = (int32_t)std::min<int64_t>(bsz, n - b0);
      a.nblk = (a.rows + 63) / 64;
      a.loss_acc = b.loss + e;
      ++step;
      a.c1 = 1.0f - powf(p->beta1, (float)step);
      a.c2 = 1.0f - powf(p->beta2, (float)step);
      launch_train_batch(a, s);
      launch_train_update(a, s);
      ++batches;
    }
    HIPCHK(hipGetLastError());
  }
  std::vector<double> lh(p->epochs);
  HIPCHK(hipMemcpyAsync(params_of(model), b.master, sizeof(float) * kNumParams,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(model->feat_mean, b.mlp->fmean, sizeof(float) * kFeat, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(model->feat_std, b.mlp->fstd, sizeof(float) * kFeat, hipMemcpyDeviceToHost, s));
  float tm[4], ts[4];
  HIPCHK(hipMemcpyAsync(tm, b.mlp->tmean, sizeof tm, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(ts, b.mlp->tstd, sizeof ts, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(lh.data(), b.loss, sizeof(double) * p->epochs, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < 3; ++k) {
    model->tgt_mean[k] = k < model->dim ? tm[k] : 0.0f;
    model->tgt_std[k] = k < model->dim ? ts[k] : 1.0f;
  }
  if (loss_hist)
    for (int e = 0; e < p->epochs; ++e) loss_hist[e] = (float)(lh[e] / (double)batches);
  return AQS_OK;
}

// ---------------------------------------------------------------------------
// Training without device allocation: the buffers of train_run live in a
// fixed device array of this library, one per GPU.

constexpr int64_t kStaticSamples = AQS_STATIC_TRAIN_MAX_SAMPLES;
constexpr int64_t kStaticBatchBlocks = (AQS_STATIC_TRAIN_MAX_BATCH + 63) / 64;
constexpr int64_t kStaticEpochs = AQS_STATIC_TRAIN_MAX_EPOCHS;

constexpr size_t al256(size_t x) { return (x + 255) / 256 * 256; }
// byte offsets of the buffers in the array
constexpr size_t kSoZ = 0;
constexpr size_t kSoT = kSoZ + al256(sizeof(uint16_t) * kFeat * kStaticSamples);
constexpr size_t kSoStats = kSoT + al256(sizeof(float) * 4 * kStaticSamples);
constexpr size_t kSoStatPart = kSoStats + al256(sizeof(double) * 2 * 68);
constexpr size_t kSoKeep = kSoStatPart + al256(sizeof(double) * 65 * 256);
constexpr size_t kSoPart = kSoKeep + al256(sizeof(uint8_t) * kStaticSamples);
constexpr size_t kSoMaster = kSoPart + al256(sizeof(float) * (size_t)(kNumParams + 1) * kStaticBatchBlocks);
constexpr size_t kSoM = kSoMaster + al256(sizeof(float) * kNumParams);
constexpr size_t kSoV = kSoM + al256(sizeof(float) * kNumParams);
constexpr size_t kSoLoss = kSoV + al256(sizeof(float) * kNumParams);
constexpr size_t kSoMlp = kSoLoss + al256(sizeof(double) * kStaticEpochs);
constexpr size_t kScratchBytes = kSoMlp + al256(sizeof(MlpDev));
static_assert(kScratchBytes == AQS_STATIC_TRAIN_SCRATCH_BYTES,
              "the header states the size of the training scratch array");

// Device addresses of the array, per device, taken once with that device
// current (the host-side name of the array is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

aqs_status scratch_address(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(AQS_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(AQS_EHIP, "hipGetSymbolAddress of the training scratch array failed: %s",
                  hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return AQS_OK;
}

}  // namespace

extern "C" {

aqs_status aqs_mlp_train(const aqs_train_params* p, int64_t n, const float* feat,
                         const float* target, const int32_t* order, aqs_mlp* model,
                         float* loss_hist, void* stream) {
  aqs_status st = check_train(p, n, feat, target, order, model);
  if (st) return st;
  const int32_t bsz = (int32_t)std::min<int64_t>(p->batch, n);
  const int32_t maxblk = (bsz + 63) / 64;
  TrainBufs b;
  st = train_alloc(b, n, maxblk, p->epochs, true);
  if (st) return st;
  return train_run(p, n, feat, target, order, model, loss_hist, (hipStream_t)stream, b);
}

aqs_status aqs_mlp_train_static(const aqs_train_params* p, int64_t n, const float* feat,
                                const float* target, const int32_t* order, aqs_mlp* model,
                                float* loss_hist, void* stream) {
  aqs_status st = check_train(p, n, feat, target, order, model);
  if (st) return st;
  if (n > kStaticSamples || std::min<int64_t>(p->batch, n) > AQS_STATIC_TRAIN_MAX_BATCH ||
      p->epochs > kStaticEpochs)
    return fail(AQS_ECAPACITY,
                "aqs_mlp_train_static holds at most %lld samples, batches of %d and %lld epochs "
                "(asked: %lld, %d, %d)",
                (long long)kStaticSamples, AQS_STATIC_TRAIN_MAX_BATCH, (long long)kStaticEpochs,
                (long long)n, p->batch, p->epochs);
  void* base = nullptr;
  st = scratch_address(&base);
  if (st) return st;
  char* w = static_cast<char*>(base);
  TrainPtrs b;
  b.z = reinterpret_cast<uint16_t*>(w + kSoZ);
  b.t = reinterpret_cast<float*>(w + kSoT);
  b.stats = reinterpret_cast<double*>(w + kSoStats);
  b.stat_part = reinterpret_cast<double*>(w + kSoStatPart);
  b.keep = reinterpret_cast<uint8_t*>(w + kSoKeep);
  b.part = reinterpret_cast<float*>(w + kSoPart);
  b.master = reinterpret_cast<float*>(w + kSoMaster);
  b.m = reinterpret_cast<float*>(w + kSoM);
  b.v = reinterpret_cast<float*>(w + kSoV);
  b.loss = reinterpret_cast<double*>(w + kSoLoss);
  b.mlp = reinterpret_cast<MlpDev*>(w + kSoMlp);
  return train_run(p, n, feat, target, order, model, loss_hist, (hipStream_t)stream, b);
}

aqs_status aqs_mlp_gradients(const aqs_mlp* model, int64_t n, const float* feat,
                             const float* target, float huber_delta, aqs_mlp* grad,
                             float* loss, void* stream) {
  if (!feat || !target || !grad) return fail(AQS_EINVAL, "null argument");
  aqs_status st = check_mlp(model);
  if (st) return st;
  if (n <= 0 || n > 65536) return fail(AQS_EINVAL, "gradient batch must hold 1..65536 samples");
  hipStream_t s = (hipStream_t)stream;
  const int32_t nblk = (int32_t)((n + 63) / 64);
  TrainBufs b;
  st = train_alloc(b, n, nblk, 1, false);
  if (st) return st;
  if (hipMalloc((void**)&b.order, sizeof(int32_t) * n) != hipSuccess)
    return fail(AQS_EHIP, "device allocation failed");
  std::vector<int32_t> iota(n);
  for (int64_t i = 0; i < n; ++i) iota[i] = (int32_t)i;
  HIPCHK(hipMemcpyAsync(b.order, iota.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(b.loss, 0, sizeof(double), s));
  st = upload_mlp(s, model, b.master, b.mlp, true);
  if (st) return st;
  TrainArgs a{};
  a.feat = feat;
  a.tgt = target;
  a.n = n;
  a.dim = model->dim;
  a.z = b.z;
  a.t = b.t;
  a.delta = huber_delta;
  a.part = b.part;
  a.mlp = b.mlp;
  a.order = b.order;
  a.b0 = 0;
  a.rows = (int32_t)n;
  a.nblk = nblk;
  a.grad_out = b.grad;
  a.loss_acc = b.loss;
  launch_train_prep(a, s);
  launch_train_batch(a, s);
  launch_train_update(a, s);
  HIPCHK(hipGetLastError());
  double lv = 0.0;
  *grad = *model;
  HIPCHK(hipMemcpyAsync(params_of(grad), b.grad, sizeof(float) * kNumParams, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&lv, b.loss, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (loss) *loss = (float)lv;
  return AQS_OK;
}

}  // extern "C"
