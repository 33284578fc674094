/* The C ABI of libaqs.so driven from plain C (no Python, no torch): a
 * Lennard-Jones dimer in a 2D periodic box minimised to the analytic
 * minimum r* = 2^(1/6) sigma_AA, E* = -1 - U(rc) (Eq. 13 with rc = 2.5),
 * then sheared and stepped (a bond along x does not feel x += gamma y), the
 * strain index and the equality test of Eq. (20) checked, and an invalid
 * call reported through aqs_last_error.  Prints "abi ok" and exits 0 on
 * success. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "aqs.h"

#define CHECK(cond, ...)                            \
  do {                                              \
    if (!(cond)) {                                  \
      fprintf(stderr, "FAIL line %d: ", __LINE__);  \
      fprintf(stderr, __VA_ARGS__);                 \
      fprintf(stderr, " (%s)\n", aqs_last_error()); \
      return 1;                                     \
    }                                               \
  } while (0)

int main(void) {
  aqs_potential pot;
  memset(&pot, 0, sizeof pot);
  pot.dim = 2;
  const double eps[2][2] = {{1.0, 1.5}, {1.5, 0.5}}, sig[2][2] = {{1.0, 0.8}, {0.8, 0.88}};
  memcpy(pot.eps, eps, sizeof eps);
  memcpy(pot.sigma, sig, sizeof sig);
  pot.rc_factor = 2.5;
  aqs_fire_params fire = {0.01, 0.03, 2e-4, 1.2, 0.9, 0.2, 0.95, 0.1, 1e-10, 5, 2000, 1, 0, 1000000};
  aqs_tuning tune;
  memset(&tune, 0, sizeof tune);
  const int32_t n_atoms[1] = {2};
  const double box[2] = {10.0, 10.0}, dgamma[1] = {1e-3};

  const size_t bytes = aqs_workspace_bytes(&pot, &tune, 1, n_atoms, box);
  CHECK(bytes > 0, "workspace size");
  void* ws = NULL;
  CHECK(hipMalloc(&ws, bytes) == hipSuccess, "hipMalloc of %zu bytes", bytes);
  aqs_ctx* ctx = NULL;
  CHECK(aqs_create(&pot, &fire, &tune, 1, n_atoms, box, dgamma, ws, bytes, NULL, &ctx) == AQS_OK,
        "aqs_create");

  const uint8_t types[2] = {0, 0};
  const double pos0[4] = {4.0, 5.0, 5.2, 5.0};
  CHECK(aqs_set_replica(ctx, 0, types, pos0, 0) == AQS_OK, "aqs_set_replica");
  const int32_t rep[1] = {0};
  aqs_step_record rec[4];
  CHECK(aqs_minimize_batch(ctx, 1, rep, AQS_START_PLAIN, NULL, NULL, rec) == AQS_OK, "minimise");
  double pos[4];
  CHECK(aqs_get_positions(ctx, 0, pos) == AQS_OK, "positions");
  const double r = hypot(pos[2] - pos[0], pos[3] - pos[1]);
  const double rstar = pow(2.0, 1.0 / 6.0);
  const double urc = 4.0 * (pow(2.5, -12.0) - pow(2.5, -6.0));
  const double estar = -1.0 - urc;
  CHECK(rec[0].status == AQS_CONVERGED, "status %d", rec[0].status);
  CHECK(fabs(r - rstar) < 1e-9, "bond %.15f against %.15f", r, rstar);
  CHECK(fabs(rec[0].energy - estar) < 1e-12, "energy %.15f against %.15f", rec[0].energy, estar);

  const int64_t dk[1] = {5};
  CHECK(aqs_affine_shear(ctx, 1, rep, dk) == AQS_OK, "affine shear");
  const int32_t steps[1] = {3};
  CHECK(aqs_minimize_batch(ctx, 1, rep, AQS_START_PLAIN, steps, NULL, rec) == AQS_OK, "chain");
  for (int s = 0; s <= 3; ++s) {
    CHECK(rec[s].status == AQS_CONVERGED, "step %d status %d", s, rec[s].status);
    CHECK(fabs(rec[s].energy - estar) < 1e-12, "step %d energy %.15f", s, rec[s].energy);
  }
  int64_t k = -1;
  CHECK(aqs_get_strain_index(ctx, 0, &k) == AQS_OK && k == 8, "strain index %lld", (long long)k);
  int32_t equal = 0;
  double md = -1.0, de = -1.0;
  CHECK(aqs_compare_configs(ctx, 0, 0, 1e-4, &equal, &md, &de) == AQS_OK && equal == 1 && md == 0.0,
        "self comparison");

  CHECK(aqs_copy_replica(ctx, 0, 5) == AQS_EINVAL, "a slot out of range is refused");
  CHECK(strlen(aqs_last_error()) > 0, "error message");

  CHECK(aqs_destroy(ctx) == AQS_OK, "destroy");
  CHECK(hipFree(ws) == hipSuccess, "hipFree");
  printf("abi ok\n");
  return 0;
}
