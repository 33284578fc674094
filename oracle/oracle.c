/*
 * oracle.c -- plain CPU FP64 reference of the AQS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the product path never
 * does.  It shares no code, header, table or constant with the GPU library.
 *
 * Method: Reihn, Bamer, Stamm, "Parallel athermal quasistatic deformation
 * stepping of molecular systems" (arXiv 2507.20802).
 *
 * Everything is the plain definition, written for a reader to check by eye:
 * O(N^2) pair sums in atom order, explicit fractional coordinates for the
 * minimum image, FP64 throughout, no FMA contraction (built with
 * -ffp-contract=off), every sum taken in a fixed order.  OpenMP only splits
 * the outer atom loop; each per-atom sum is still taken j = 0..N-1 and the
 * per-atom results are combined sequentially in atom order.
 *
 * Conventions
 *   pos    atom-major, pos[i*dim + a], a = x, y (, z)
 *   H      dim x dim, row-major, columns are the Bravais vectors h_1..h_d
 *          (Sec. 2.1, "Formalism"); simple shear keeps H upper triangular,
 *          the pure shear of Eq. (17) gives a general (x, y) block
 *   type   0 (A) or 1 (B)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t pad_;
  double eps[2][2];     /* bond strength epsilon_ab, Eq. (13) */
  double sigma[2][2];   /* zero-energy distance sigma_ab, Eq. (13) */
  double rc_factor;     /* cutoff radius of pair ab = rc_factor * sigma_ab */
} orc_pot;

typedef struct {
  double dt0, dt_max, dt_min, f_inc, f_dec, alpha0, f_alpha, dmax, ftol;
  int32_t n_delay, n_neg_max, initial_delay, pad_;
  int64_t max_iter;
} orc_fire_params;

enum { ORC_CONVERGED = 0, ORC_MAXITER = 1, ORC_STALLED = 2, ORC_NONFINITE = 3 };

/* ------------------------------------------------------------------------ */
/* threads                                                                   */

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Lennard-Jones pair, Eq. (13), truncated at rc_ab and shifted so that the
 * energy is continuous (zero) at the cutoff; the force is not shifted, so the
 * dimer minimum stays at 2^(1/6) sigma.  The per-type-pair constants are
 * tabulated once per call (cutoff^2, sigma^2, 4 eps, energy at the cutoff).
 */
typedef struct {
  double rc2[2][2], sig2[2][2], eps4[2][2], ucut[2][2];
} pair_table;

static void make_table(const orc_pot* p, pair_table* t) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const double sig = p->sigma[a][b], eps = p->eps[a][b];
      const double rc = p->rc_factor * sig;
      const double sc2 = (sig * sig) / (rc * rc);
      const double sc6 = sc2 * sc2 * sc2;
      t->rc2[a][b] = rc * rc;
      t->sig2[a][b] = sig * sig;
      t->eps4[a][b] = 4.0 * eps;
      t->ucut[a][b] = 4.0 * eps * (sc6 * sc6 - sc6);
    }
}

/* Returns 1 if r2 < rc^2 and sets *u = U(r) - U(rc), *g = U'(r) / r.        */
static inline int pair_lj(const pair_table* t, int ti, int tj, double r2,
                          double* u, double* g) {
  if (!(r2 < t->rc2[ti][tj])) return 0;
  const double sr2 = t->sig2[ti][tj] / r2;
  const double sr6 = sr2 * sr2 * sr2;
  const double sr12 = sr6 * sr6;
  *u = t->eps4[ti][tj] * (sr12 - sr6) - t->ucut[ti][tj];
  /* dU/dr = 4 eps (-12 sigma^12 r^-13 + 6 sigma^6 r^-7); divide by r */
  *g = t->eps4[ti][tj] * (-12.0 * sr12 + 6.0 * sr6) / r2;
  return 1;
}

/* Public for tests: the single pair terms. */
int orc_pair(const orc_pot* p, int ti, int tj, double r2, double* u, double* g) {
  pair_table t;
  make_table(p, &t);
  *u = 0.0;
  *g = 0.0;
  return pair_lj(&t, ti, tj, r2, u, g);
}

/* ------------------------------------------------------------------------ */
/* box geometry                                                              */

static int upper_triangular(int dim, const double* H) {
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < a; ++b)
      if (H[a * dim + b] != 0.0) return 0;
  return 1;
}

/* The boxes here: upper triangular (simple shear), or a general (x, y)
 * block with z neutral (the pure shear of Eq. 17, whose map also has a
 * lower off-diagonal entry).  A z coupling is not supported.               */
static int supported_box(int dim, const double* H) {
  if (dim == 2) return 1;
  return H[2] == 0.0 && H[5] == 0.0 && H[6] == 0.0 && H[7] == 0.0;
}

/* inverse of an upper-triangular matrix by back substitution */
static void inv_upper(int dim, const double* H, double* Hi) {
  memset(Hi, 0, sizeof(double) * dim * dim);
  for (int c = 0; c < dim; ++c) {
    /* solve H x = e_c */
    double x[3] = {0, 0, 0};
    for (int a = dim - 1; a >= 0; --a) {
      double t = (a == c) ? 1.0 : 0.0;
      for (int b = a + 1; b < dim; ++b) t -= H[a * dim + b] * x[b];
      x[a] = t / H[a * dim + a];
    }
    for (int a = 0; a < dim; ++a) Hi[a * dim + c] = x[a];
  }
}

static double det_upper(int dim, const double* H) {
  double d = 1.0;
  for (int a = 0; a < dim; ++a) d *= H[a * dim + a];
  return d;
}

/* Inverse and determinant of a supported box: back substitution when upper
 * triangular, else the 2x2 (x, y) block by its adjugate (and 1/Lz).         */
static void inv_box(int dim, const double* H, double* Hi) {
  if (upper_triangular(dim, H)) {
    inv_upper(dim, H, Hi);
    return;
  }
  memset(Hi, 0, sizeof(double) * dim * dim);
  const double a = H[0], b = H[1], c = H[dim], d = H[dim + 1];
  const double det = a * d - b * c;
  Hi[0] = d / det;
  Hi[1] = -b / det;
  Hi[dim] = -c / det;
  Hi[dim + 1] = a / det;
  if (dim == 3) Hi[8] = 1.0 / H[8];
}

static double det_box(int dim, const double* H) {
  if (upper_triangular(dim, H)) return det_upper(dim, H);
  const double d2 = H[0] * H[dim + 1] - H[1] * H[dim];
  return dim == 3 ? d2 * H[8] : d2;
}

/* Perpendicular widths of the cell spanned by the columns of H: the distance
 * between the two faces that do not contain h_a, i.e. |det H| / |area of the
 * other vectors|.                                                           */
void orc_perp_widths(int dim, const double* H, double* w) {
  double vol = fabs(det_box(dim, H));
  if (dim == 2) {
    double h0 = sqrt(H[0] * H[0] + H[2] * H[2]);
    double h1 = sqrt(H[1] * H[1] + H[3] * H[3]);
    w[0] = vol / h1;
    w[1] = vol / h0;
    return;
  }
  for (int a = 0; a < 3; ++a) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    double u[3], v[3], x[3];
    for (int k = 0; k < 3; ++k) {
      u[k] = H[k * 3 + b];
      v[k] = H[k * 3 + c];
    }
    x[0] = u[1] * v[2] - u[2] * v[1];
    x[1] = u[2] * v[0] - u[0] * v[2];
    x[2] = u[0] * v[1] - u[1] * v[0];
    w[a] = vol / sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  }
}

/* Minimum image of a difference vector under the periodic lattice H
 * (Sec. 2.1: periodic boundaries along every Bravais vector): go to
 * fractional coordinates, subtract the nearest integer, go back.            */
static inline __attribute__((always_inline)) void min_image(int dim, const double* H, const double* Hi, double* d) {
  double s[3];
  for (int a = 0; a < dim; ++a) {
    double t = 0.0;
    for (int b = 0; b < dim; ++b) t += Hi[a * dim + b] * d[b];
    s[a] = t - nearbyint(t);
  }
  for (int a = 0; a < dim; ++a) {
    double t = 0.0;
    for (int b = 0; b < dim; ++b) t += H[a * dim + b] * s[b];
    d[a] = t;
  }
}

static double rc_max(const orc_pot* p) {
  double m = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      if (p->rc_factor * p->sigma[a][b] > m) m = p->rc_factor * p->sigma[a][b];
  return m;
}

/* 1 if the minimum image is exact for this cutoff (rc < half the smallest
 * perpendicular width), else 0.                                             */
int orc_min_image_valid(int dim, const double* H, const orc_pot* p) {
  double w[3];
  orc_perp_widths(dim, H, w);
  double wmin = w[0];
  for (int a = 1; a < dim; ++a)
    if (w[a] < wmin) wmin = w[a];
  return rc_max(p) < 0.5 * wmin;
}

/* Sum over j of the pair terms of atom i, minimum image (mode 0).  The pair
 * energy and stress of i<j go to i; the force on i takes every j != i.
 * D is a compile-time 2 or 3 after inlining.                                 */
static inline __attribute__((always_inline)) void atom_sum_min_image(
    const int D, int i, int n, const double* pos, const uint8_t* type,
    const double* H, const double* Hi, const pair_table* tab, double* f,
    double* e, double* s) {
  const int ti = type[i];
  for (int j = 0; j < n; ++j) {
    if (j == i) continue;
    double d[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) d[a] = pos[j * D + a] - pos[i * D + a];
    min_image(D, H, Hi, d);
    double r2 = 0.0;
    for (int a = 0; a < D; ++a) r2 += d[a] * d[a];
    double u, g;
    if (!pair_lj(tab, ti, type[j], r2, &u, &g)) continue;
    for (int a = 0; a < D; ++a) f[a] += g * d[a];
    if (j > i) {
      *e += u;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) s[a * 3 + b] += g * d[a] * d[b];
    }
  }
}

/* Sum over j and over lattice translations H n, n in [-m, m]^dim, of the pair
 * terms of atom i (mode 1); half of each ordered pair's energy and stress.  */
static void atom_sum_images(int dim, int i, int n, const double* pos,
                            const uint8_t* type, const double* H, int m,
                            const pair_table* tab, double* f, double* e,
                            double* s) {
  int nimg = 1;
  for (int a = 0; a < dim; ++a) nimg *= (2 * m + 1);
  const int ti = type[i];
  for (int j = 0; j < n; ++j) {
    for (int k = 0; k < nimg; ++k) {
      int nn[3] = {0, 0, 0}, kk = k;
      for (int a = 0; a < dim; ++a) {
        nn[a] = kk % (2 * m + 1) - m;
        kk /= (2 * m + 1);
      }
      if (j == i && nn[0] == 0 && nn[1] == 0 && nn[2] == 0) continue;
      double d[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) {
        double t = pos[j * dim + a] - pos[i * dim + a];
        for (int b = 0; b < dim; ++b) t += H[a * dim + b] * (double)nn[b];
        d[a] = t;
      }
      double r2 = 0.0;
      for (int a = 0; a < dim; ++a) r2 += d[a] * d[a];
      double u, g;
      if (!pair_lj(tab, ti, type[j], r2, &u, &g)) continue;
      for (int a = 0; a < dim; ++a) f[a] += g * d[a];
      *e += 0.5 * u;
      for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) s[a * 3 + b] += 0.5 * g * d[a] * d[b];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Energy, forces and stress.
 *
 *   E          = sum_{i<j} U(r_ij)                                  (Eq. 4)
 *   F_i        = -dE/dr_i = sum_{j != i} U'(r_ij) d_ij / r_ij,
 *                d_ij = r_j - r_i (minimum image)                    (Eq. 6)
 *   sigma_ab   = (1/V) sum_{i<j} U'(r_ij) d_a d_b / r_ij
 *                (sigma_xy V is dE/dgamma under affine simple shear of the
 *                Lagrangian energy, Eq. 5; tau = sigma_12 of Fig. 2)
 *
 * image_mode 0: minimum image (requires orc_min_image_valid).
 * image_mode 1: explicit sum over lattice translations H n, n in
 *               [-image_range, image_range]^dim, every pair (i, j, n) except
 *               (i, i, 0); energies and stresses take half of each ordered
 *               pair.  Valid for any box; used to pin mode 0.
 *
 * Outputs (any may be NULL): E, F[n*dim], S[dim*dim] (stress), e_atom[n]
 * (energy of pairs i<j assigned to i in mode 0; half of every pair of i in
 * mode 1).  Returns 0, or -1 if H is not upper triangular, or -2 if mode 0
 * is requested for a box that is too small.                                 */
int orc_eval(int dim, int n, const double* pos, const uint8_t* type,
             const double* H, const orc_pot* p, int image_mode,
             int image_range, double* E, double* F, double* S,
             double* e_atom) {
  if (!supported_box(dim, H)) return -1;
  if (image_mode == 0 && !orc_min_image_valid(dim, H, p)) return -2;
  double Hi[9];
  inv_box(dim, H, Hi);
  const double vol = fabs(det_box(dim, H));
  pair_table tab;
  make_table(p, &tab);

  double* ei = (double*)calloc((size_t)n, sizeof(double));
  double* si = (double*)calloc((size_t)n * 9, sizeof(double));
  double* fi = (double*)calloc((size_t)n * dim, sizeof(double));

  const int m = image_range;

#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    double f[3] = {0, 0, 0};
    double e = 0.0;
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (image_mode == 0) {
      if (dim == 2)
        atom_sum_min_image(2, i, n, pos, type, H, Hi, &tab, f, &e, s);
      else
        atom_sum_min_image(3, i, n, pos, type, H, Hi, &tab, f, &e, s);
    } else {
      atom_sum_images(dim, i, n, pos, type, H, m, &tab, f, &e, s);
    }
    ei[i] = e;
    for (int a = 0; a < dim; ++a) fi[i * dim + a] = f[a];
    for (int a = 0; a < 9; ++a) si[(size_t)i * 9 + a] = s[a];
  }

  double etot = 0.0, stot[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    etot += ei[i];
    for (int a = 0; a < 9; ++a) stot[a] += si[(size_t)i * 9 + a];
  }
  if (E) *E = etot;
  if (F) memcpy(F, fi, sizeof(double) * (size_t)n * dim);
  if (S)
    for (int a = 0; a < dim; ++a)
      for (int b = 0; b < dim; ++b) S[a * dim + b] = stot[a * 3 + b] / vol;
  if (e_atom) memcpy(e_atom, ei, sizeof(double) * (size_t)n);
  free(ei);
  free(si);
  free(fi);
  return 0;
}

/* Forces on a chosen subset of atoms only, each computed one by one with the
 * full O(N) minimum-image sum (for sampled checks at large N).              */
int orc_forces_on(int dim, int n, const double* pos, const uint8_t* type,
                  const double* H, const orc_pot* p, int nsel,
                  const int64_t* sel, double* F) {
  if (!supported_box(dim, H)) return -1;
  if (!orc_min_image_valid(dim, H, p)) return -2;
  double Hi[9];
  inv_box(dim, H, Hi);
  pair_table tab;
  make_table(p, &tab);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < nsel; ++k) {
    const int64_t i = sel[k];
    double f[3] = {0, 0, 0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) d[a] = pos[j * dim + a] - pos[i * dim + a];
      min_image(dim, H, Hi, d);
      double r2 = 0.0;
      for (int a = 0; a < dim; ++a) r2 += d[a] * d[a];
      double u, g;
      if (!pair_lj(&tab, type[i], type[j], r2, &u, &g)) continue;
      for (int a = 0; a < dim; ++a) f[a] += g * d[a];
    }
    for (int a = 0; a < dim; ++a) F[k * dim + a] = f[a];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Affine simple shear of the atom positions, Eqs. (2)-(3) with the matrix of
 * Eq. (16): x_i <- x_i + dgamma * y_i.  In 3D the same map acts on (x, y)
 * and leaves z alone.  The caller updates the box H <- F H.                 */
void orc_affine(int dim, int n, double* pos, double dgamma) {
  for (int i = 0; i < n; ++i) pos[i * dim + 0] += dgamma * pos[i * dim + 1];
}

/* A general linear map of (x, y), z unchanged: r_i <- M r_i with M row-major
 * 2x2 (the pure shear of Eq. 17 and its powers).                            */
void orc_linear_xy(int dim, int n, double* pos, const double* M) {
  for (int i = 0; i < n; ++i) {
    const double x = pos[i * dim + 0], y = pos[i * dim + 1];
    pos[i * dim + 0] = M[0] * x + M[1] * y;
    pos[i * dim + 1] = M[2] * x + M[3] * y;
  }
}

/* ------------------------------------------------------------------------ */
/* The minimisation operator of Eq. (10), realised by FIRE 2.0 (Guenole et
 * al., Comput. Mater. Sci. 173 (2020) 109584, semi-implicit Euler form) in
 * place of the paper's conjugate gradients.  Unit mass.  Steps, in order:
 *
 *   1  evaluate E, F at x
 *   2  if the energy, a force or a position is not finite: NONFINITE
 *      if max_i |F_i| < ftol: CONVERGED (checked before any update, so an
 *      inherent structure takes zero iterations)
 *   3  P = F . v
 *   4  P > 0:  n_pos += 1, n_neg = 0; if n_pos > n_delay:
 *              dt = min(dt f_inc, dt_max), alpha *= f_alpha
 *   5  P <= 0: n_pos = 0, n_neg += 1; if n_neg > n_neg_max: STALLED;
 *              unless (initial_delay and it < n_delay):
 *                  if dt f_dec >= dt_min: dt *= f_dec;  alpha = alpha0
 *              x -= dt v / 2;  v = 0
 *   6  v += dt F
 *   7  v = (1 - alpha) v + alpha (|v| / |F|) F   (global 2-norms after 6;
 *      skipped if |F| = 0)
 *   8  per atom: if dt |v_i| > dmax, scale v_i to dt |v_i| = dmax
 *   9  x += dt v;  it += 1;  if it >= max_iter: MAXITER
 *
 * On return pos holds the final positions; E and fmax are those of the last
 * force evaluation.  trace_E (optional) receives the energy of every
 * evaluation, up to trace_cap entries.                                      */
int orc_fire(int dim, int n, double* pos, const uint8_t* type, const double* H,
             const orc_pot* p, const orc_fire_params* fp, int64_t* iters,
             double* E_out, double* fmax_out, int32_t* status,
             double* trace_E, int64_t trace_cap) {
  const size_t nd = (size_t)n * dim;
  double* v = (double*)calloc(nd, sizeof(double));
  double* F = (double*)calloc(nd, sizeof(double));
  double dt = fp->dt0, alpha = fp->alpha0, E = 0.0, fmax = 0.0;
  int64_t it = 0, n_pos = 0, n_neg = 0;
  int st = ORC_MAXITER, rc = 0;
  for (;;) {
    rc = orc_eval(dim, n, pos, type, H, p, 0, 0, &E, F, NULL, NULL);
    if (rc != 0) break;
    fmax = 0.0;
    int finite = isfinite(E);
    for (size_t k = 0; k < nd; ++k)
      if (!isfinite(pos[k])) finite = 0;
    for (int i = 0; i < n; ++i) {
      double f2 = 0.0;
      for (int a = 0; a < dim; ++a) f2 += F[i * dim + a] * F[i * dim + a];
      double fi = sqrt(f2);
      if (!isfinite(fi)) finite = 0;
      if (fi > fmax) fmax = fi;
    }
    if (trace_E && it < trace_cap) trace_E[it] = E;
    if (!finite) {
      st = ORC_NONFINITE;
      break;
    }
    if (fmax < fp->ftol) {
      st = ORC_CONVERGED;
      break;
    }
    double P = 0.0;
    for (size_t k = 0; k < nd; ++k) P += F[k] * v[k];
    if (P > 0.0) {
      n_pos += 1;
      n_neg = 0;
      if (n_pos > fp->n_delay) {
        dt = fmin(dt * fp->f_inc, fp->dt_max);
        alpha *= fp->f_alpha;
      }
    } else {
      n_pos = 0;
      n_neg += 1;
      if (n_neg > fp->n_neg_max) {
        st = ORC_STALLED;
        break;
      }
      if (!(fp->initial_delay && it < fp->n_delay)) {
        if (dt * fp->f_dec >= fp->dt_min) dt *= fp->f_dec;
        alpha = fp->alpha0;
      }
      for (size_t k = 0; k < nd; ++k) {
        pos[k] -= 0.5 * dt * v[k];
        v[k] = 0.0;
      }
    }
    for (size_t k = 0; k < nd; ++k) v[k] += dt * F[k];
    double vv = 0.0, ff = 0.0;
    for (size_t k = 0; k < nd; ++k) {
      vv += v[k] * v[k];
      ff += F[k] * F[k];
    }
    if (ff > 0.0) {
      const double c = alpha * sqrt(vv) / sqrt(ff);
      for (size_t k = 0; k < nd; ++k) v[k] = (1.0 - alpha) * v[k] + c * F[k];
    }
    for (int i = 0; i < n; ++i) {
      double v2 = 0.0;
      for (int a = 0; a < dim; ++a) v2 += v[i * dim + a] * v[i * dim + a];
      const double step = dt * sqrt(v2);
      if (step > fp->dmax) {
        const double sc = fp->dmax / step;
        for (int a = 0; a < dim; ++a) v[i * dim + a] *= sc;
      }
    }
    for (size_t k = 0; k < nd; ++k) pos[k] += dt * v[k];
    it += 1;
    if (it >= fp->max_iter) {
      st = ORC_MAXITER;
      break;
    }
  }
  free(v);
  free(F);
  if (iters) *iters = it;
  if (E_out) *E_out = E;
  if (fmax_out) *fmax_out = fmax;
  if (status) *status = st;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* The minimisation operator of Eq. (10) by nonlinear conjugate gradients,
 * the minimiser the paper itself uses (Sec. 2.1).  The paper names the method
 * only; this is the Polak-Ribiere variant with non-negative beta (automatic
 * restart) and a line search that needs forces only: it walks along the
 * direction d to the first point where the directional derivative
 * phi'(a) = -F(x0 + a d) . d changes sign (the nearest minimum along d, in
 * keeping with the search for the adjacent minimum of Eq. (9)).
 *
 * One force evaluation per iteration.  State of a line search: origin
 * derivative p0 = phi'(0) < 0, trial step a, the last point still descending
 * (a_lo, p_lo) and, once found, the first point past the minimum
 * (a_hi, p_hi).  Steps, in order, at every evaluation:
 *
 *   1  evaluate E, F at x
 *   2  if the energy, a force or a position is not finite: NONFINITE
 *      if max_i |F_i| < ftol: CONVERGED (before any update)
 *   3  with a direction: p = -F . d, dn = max_i |d_i|, a_max = dmax / dn;
 *      the line search ends if |p| <= sigma |p0| (the curvature condition of
 *      strong Wolfe) or if p < 0 with a >= a_max (the displacement cap);
 *      then beta = max(0, (|F|^2 - F . F_0) / |F_0|^2), F_0 the force at the
 *      origin (Polak-Ribiere, non-negative), and a new direction follows (6)
 *   4  otherwise one more evaluation in this line search; after ls_max of
 *      them the search has failed: beta = 0 (steepest descent from x, 6) and,
 *      after more than n_fail_max consecutive failures, STALLED
 *   5  next trial: p < 0 -> (a_lo, p_lo) = (a, p), else (a_hi, p_hi) = (a, p);
 *      no upper point yet: the secant through the previous and the new lower
 *      point extrapolates, a' = a - p (a - a_lo_prev) / (p - p_lo_prev),
 *      clamped to [1.1 a, grow a] (grow a if p <= p_lo_prev), then to a_max;
 *      with an upper point: the secant root between the lower and the upper
 *      point, clamped to the middle 80 % of the bracket; x += (a' - a) d
 *   6  new direction: F . (F + beta d) = |F|^2 - beta p; if it is not
 *      positive, beta = 0;  d = F + beta d (d = F if beta = 0);
 *      p0 = -F . d; first trial a1 = a_prev p0_prev / p0 (the previous
 *      search's accepted step a_prev and origin derivative p0_prev), or
 *      a_init for the first search and after a failed one, capped at
 *      dmax / (max_i |F_i| + beta dn) so that no atom moves more than dmax;
 *      F_0 = F; x += a1 d
 *   7  it += 1; if it >= max_iter: MAXITER
 *
 * The core takes the force field as a callback (the tests also run it on a
 * quadratic); orc_cg applies it to the Lennard-Jones system.  On return x
 * holds the final positions; E and fmax are those of the last evaluation.  */
typedef struct {
  double a_init, sigma, grow, dmax, ftol;
  int32_t ls_max, n_fail_max;
  int64_t max_iter;
} orc_cg_params;

typedef int (*orc_force_fn)(void* ctx, const double* x, double* F, double* E);

static int cg_core(int dim, int n, double* x, orc_force_fn fn, void* ctx,
                   const orc_cg_params* cp, int64_t* iters, int64_t* n_dirs,
                   double* E_out, double* fmax_out, int32_t* status) {
  const size_t nd = (size_t)n * dim;
  double* F = (double*)calloc(nd, sizeof(double));
  double* F0 = (double*)calloc(nd, sizeof(double));
  double* d = (double*)calloc(nd, sizeof(double));
  double E = 0.0, fm = 0.0;
  int have_dir = 0;
  double a = 0.0, a_lo = 0.0, p_lo = 0.0, a_hi = -1.0, p_hi = 0.0, p0 = 0.0, ff0 = 0.0;
  double a_prev = 0.0, p0_prev = 0.0;
  int64_t it = 0, dirs = 0, nls = 0, nfail = 0;
  int st = ORC_MAXITER, rc = 0;
  for (;;) {
    rc = fn(ctx, x, F, &E);                                  /* 1 */
    if (rc != 0) break;
    int finite = isfinite(E);                                /* 2 */
    for (size_t k = 0; k < nd; ++k)
      if (!isfinite(x[k])) finite = 0;
    fm = 0.0;
    for (int i = 0; i < n; ++i) {
      double f2 = 0.0;
      for (int c = 0; c < dim; ++c) f2 += F[i * dim + c] * F[i * dim + c];
      const double fi = sqrt(f2);
      if (!isfinite(fi)) finite = 0;
      if (fi > fm) fm = fi;
    }
    if (!finite) {
      st = ORC_NONFINITE;
      break;
    }
    if (fm < cp->ftol) {
      st = ORC_CONVERGED;
      break;
    }
    double ff = 0.0;
    for (size_t k = 0; k < nd; ++k) ff += F[k] * F[k];
    double beta = 0.0, p = 0.0, dn = 0.0;
    if (have_dir) {                                          /* 3 */
      for (size_t k = 0; k < nd; ++k) p -= F[k] * d[k];
      for (int i = 0; i < n; ++i) {
        double d2 = 0.0;
        for (int c = 0; c < dim; ++c) d2 += d[i * dim + c] * d[i * dim + c];
        if (sqrt(d2) > dn) dn = sqrt(d2);
      }
      const double a_max = cp->dmax / dn;
      if (fabs(p) <= cp->sigma * fabs(p0) || (p < 0.0 && a >= a_max)) {
        double fg = 0.0;
        for (size_t k = 0; k < nd; ++k) fg += F[k] * F0[k];
        beta = fmax(0.0, (ff - fg) / ff0);
        a_prev = a;
        p0_prev = p0;
        nfail = 0;
      } else if (++nls > cp->ls_max) {                       /* 4 */
        if (++nfail > cp->n_fail_max) {
          st = ORC_STALLED;
          break;
        }
        a_prev = 0.0;
      } else {                                               /* 5 */
        const double a_old = a_lo, p_old = p_lo;
        if (p < 0.0) {
          a_lo = a;
          p_lo = p;
        } else {
          a_hi = a;
          p_hi = p;
        }
        double an;
        if (a_hi < 0.0) {
          an = cp->grow * a;
          if (p > p_old) an = fmin(fmax(a - p * (a - a_old) / (p - p_old), 1.1 * a), cp->grow * a);
          an = fmin(an, a_max);
        } else {
          const double w = a_hi - a_lo;
          an = fmin(fmax(a_lo - p_lo * w / (p_hi - p_lo), a_lo + 0.1 * w), a_hi - 0.1 * w);
        }
        for (size_t k = 0; k < nd; ++k) x[k] += (an - a) * d[k];
        a = an;
        it += 1;                                             /* 7 */
        if (it >= cp->max_iter) {
          st = ORC_MAXITER;
          break;
        }
        continue;
      }
    }
    double fd = ff - beta * p;                               /* 6 */
    if (!(fd > 0.0)) beta = 0.0;
    if (beta == 0.0) fd = ff;
    double a1 = (a_prev > 0.0) ? a_prev * p0_prev / (-fd) : cp->a_init;
    const double cap = cp->dmax / (fm + beta * dn);
    if (a1 > cap) a1 = cap;
    for (size_t k = 0; k < nd; ++k) {
      d[k] = (beta == 0.0) ? F[k] : F[k] + beta * d[k];
      F0[k] = F[k];
      x[k] += a1 * d[k];
    }
    p0 = -fd;
    ff0 = ff;
    a = a1;
    a_lo = 0.0;
    p_lo = p0;
    a_hi = -1.0;
    nls = 0;
    have_dir = 1;
    dirs += 1;
    it += 1;                                                 /* 7 */
    if (it >= cp->max_iter) {
      st = ORC_MAXITER;
      break;
    }
  }
  free(F);
  free(F0);
  free(d);
  if (iters) *iters = it;
  if (n_dirs) *n_dirs = dirs;
  if (E_out) *E_out = E;
  if (fmax_out) *fmax_out = fm;
  if (status) *status = st;
  return rc;
}

typedef struct {
  int dim, n;
  const uint8_t* type;
  const double* H;
  const orc_pot* p;
} lj_system;

static int lj_forces(void* ctx, const double* x, double* F, double* E) {
  const lj_system* s = (const lj_system*)ctx;
  return orc_eval(s->dim, s->n, x, s->type, s->H, s->p, 0, 0, E, F, NULL, NULL);
}

int orc_cg(int dim, int n, double* pos, const uint8_t* type, const double* H,
           const orc_pot* p, const orc_cg_params* cp, int64_t* iters, int64_t* n_dirs,
           double* E, double* fmax, int32_t* status) {
  lj_system s = {dim, n, type, H, p};
  return cg_core(dim, n, pos, lj_forces, &s, cp, iters, n_dirs, E, fmax, status);
}

/* E = sum_k kk_k x_k^2 / 2, F = -kk x: a test problem with a closed-form
 * behaviour (exact secant line searches; finite termination of CG).       */
typedef struct {
  size_t nd;
  const double* kk;
} quad_system;

static int quad_forces(void* ctx, const double* x, double* F, double* E) {
  const quad_system* q = (const quad_system*)ctx;
  double e = 0.0;
  for (size_t k = 0; k < q->nd; ++k) {
    F[k] = -q->kk[k] * x[k];
    e += 0.5 * q->kk[k] * x[k] * x[k];
  }
  *E = e;
  return 0;
}

int orc_cg_quadratic(int dim, int n, double* x, const double* kk, const orc_cg_params* cp,
                     int64_t* iters, int64_t* n_dirs, double* E, double* fmax,
                     int32_t* status) {
  quad_system q = {(size_t)n * dim, kk};
  return cg_core(dim, n, x, quad_forces, &q, cp, iters, n_dirs, E, fmax, status);
}

/* ------------------------------------------------------------------------ */
/* Configuration comparison for the equality test of Eq. (20): largest
 * minimum-image displacement between the same atom in two configurations of
 * the same box, and the mean displacement vector (a rigid-translation check).*/
int orc_compare(int dim, int n, const double* a, const double* b,
                const double* H, double* max_disp, double* mean_disp) {
  if (!supported_box(dim, H)) return -1;
  double Hi[9];
  inv_box(dim, H, Hi);
  double m = 0.0, mean[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i) {
    double d[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) d[k] = a[i * dim + k] - b[i * dim + k];
    min_image(dim, H, Hi, d);
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) {
      r2 += d[k] * d[k];
      mean[k] += d[k];
    }
    double r = sqrt(r2);
    if (r > m) m = r;
  }
  if (max_disp) *max_disp = m;
  if (mean_disp)
    for (int k = 0; k < dim; ++k) mean_disp[k] = mean[k] / (double)n;
  return 0;
}
