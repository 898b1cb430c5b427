/*
 * The C ABI without Python: register two labelled point clouds and print the
 * pose.  Two views of three orthogonal planes (the room-corner case), the
 * target moved by a known rigid motion; the registration recovers it.  Then
 * the same registration as four tickets of the batching scheduler
 * (cvo_submit / cvo_poll): each equals the synchronous result bit for bit.
 *
 *   gcc -O2 -I include register_planes.c -L paper_1904_02266_amd/lib -lcvo -lm \
 *       -Wl,-rpath,<repo>/paper_1904_02266_amd/lib -o register_planes
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "cvo.h"

static unsigned long long rng_state = 88172645463325252ull;
static double urand(void) { /* xorshift64* in [0, 1) */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
  const int n = 1500;
  float* sx = malloc(sizeof(float) * 3 * n);
  float* tx = malloc(sizeof(float) * 3 * n);
  float* lab = malloc(sizeof(float) * 5 * n);
  /* the motion that maps source points to target points: 3 deg about z,
     (0.03, -0.02, 0.01) m */
  const double a = 3.0 * M_PI / 180.0, c = cos(a), s = sin(a);
  const double M[3][4] = {{c, -s, 0, 0.03}, {s, c, 0, -0.02}, {0, 0, 1, 0.01}};
  for (int i = 0; i < n; i++) {
    double p[3];
    const int face = i % 3;
    for (int k = 0; k < 3; k++) p[k] = -2.0 + 4.0 * urand();
    p[face] = -2.0;
    for (int k = 0; k < 3; k++) sx[3 * i + k] = (float)p[k];
    for (int r = 0; r < 3; r++) tx[3 * i + r] = (float)(M[r][0] * p[0] + M[r][1] * p[1] + M[r][2] * p[2] + M[r][3]);
    for (int f = 0; f < 5; f++) lab[5 * i + f] = (float)(0.5 + 0.5 * sin(1.3 * (f + 1) * p[(f + 1) % 3] + f));
  }
  cvo_ctx* ctx = NULL;
  int rc = cvo_create(0, 0, 16, &ctx);
  if (rc) {
    fprintf(stderr, "cvo_create: %s\n", cvo_strerror(rc));
    return 1;
  }
  const cvo_cloud src = {n, 5, sx, lab, 0}, tgt = {n, 5, tx, lab, 0};
  const double ell[1] = {0.1};
  cvo_params prm = {0};
  prm.sigma = 0.1;
  prm.feat_scale = 0.2;
  prm.a2 = -1.0;
  prm.b2 = 1.0;
  prm.eta = 1.0;
  prm.cutoff_mult = 3.0;
  prm.n_stages = 1;
  prm.stage_ell = ell;
  prm.max_iters = 60;
  prm.precision = CVO_FP32_KAHAN;
  prm.step_rule = CVO_STEP_FIXED;
  const double T0[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
  double T[16];
  cvo_result res;
  rc = cvo_register(ctx, &src, &tgt, &prm, T0, T, &res);
  if (rc) {
    fprintf(stderr, "cvo_register: %s (%s)\n", cvo_strerror(rc), cvo_last_error(ctx));
    cvo_destroy(ctx);
    return 1;
  }
  /* T maps target points onto source points: T ~ M^-1 */
  const double angle = atan2(T[4], T[0]) * 180.0 / M_PI;
  printf("iterations %d F %.6f rotation about z %.4f deg translation %.4f %.4f %.4f\n", res.iters, res.F, angle,
         T[3], T[7], T[11]);

  /* the same request four times through the scheduler (host inputs are
     copied before cvo_submit returns) */
  enum { kTickets = 4 };
  uint64_t tickets[kTickets];
  for (int k = 0; k < kTickets; k++) {
    rc = cvo_submit(ctx, &src, &tgt, &prm, T0, &tickets[k]);
    if (rc) {
      fprintf(stderr, "cvo_submit: %s\n", cvo_strerror(rc));
      cvo_destroy(ctx);
      return 1;
    }
  }
  int equal = 0;
  for (int k = 0; k < kTickets; k++) {
    double Tk[16];
    cvo_result rk;
    rc = cvo_poll(ctx, tickets[k], -1, Tk, &rk);
    if (rc) {
      fprintf(stderr, "cvo_poll: %s\n", cvo_strerror(rc));
      cvo_destroy(ctx);
      return 1;
    }
    int same = rk.iters == res.iters && rk.F == res.F;
    for (int q = 0; q < 16; q++) same = same && Tk[q] == T[q];
    equal += same;
  }
  cvo_serving_counters st;
  cvo_serving_stats(ctx, &st);
  printf("served %d of %d equal to the synchronous result; completed %lld failed %lld\n", equal, kTickets,
         (long long)st.completed, (long long)st.failed);
  cvo_destroy(ctx);
  free(sx);
  free(tx);
  free(lab);
  return 0;
}
