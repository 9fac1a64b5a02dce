/*
 * Driver that runs the FP64 C oracle (oracle/coracle.c, compiled into this
 * translation unit) under AddressSanitizer and UndefinedBehaviorSanitizer; built
 * and run by tests/test_coracle.py on the CPU.  Usage: nx ny steps n_sub.
 * Seeded pseudo-random fields (xorshift64), a few coupled steps, then a read-back
 * of every field, which must be finite; prints "ok" on success.
 */
#include <stdio.h>

#include "../oracle/coracle.c"

static unsigned long long rng_state = 88172645463325252ULL;
static double urand(void) {
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (double)(rng_state >> 11) / 9007199254740992.0;
}

int main(int argc, char** argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: %s nx ny steps n_sub\n", argv[0]);
    return 2;
  }
  const int nx = atoi(argv[1]), ny = atoi(argv[2]), steps = atoi(argv[3]), n_sub = atoi(argv[4]);
  const int n = nx * ny;
  /* the small-grid parameter set with stronger drag, flow alignment and activity */
  oc_params p = {nx, ny, n_sub, 1.0, 0.8, 1.3, 0.2, 0.04, 0.04, 0.1, 0.0, 0.6, 0.04, 0.9, 0.34, 0.02};
  double* in = malloc(sizeof(double) * 7 * (size_t)n);
  double* out = malloc(sizeof(double) * 11 * (size_t)n);
  if (!in || !out) return 3;
  for (int i = 0; i < n; ++i) {
    const double th = 3.14159265358979323846 * urand();
    in[i] = 0.3 * (2.0 * urand() - 1.0);
    in[n + i] = 0.2 * cos(2.0 * th);
    in[2 * n + i] = 0.2 * sin(2.0 * th);
  }
  for (int i = 3 * n; i < 7 * n; ++i) in[i] = 2e-3 * (2.0 * urand() - 1.0);
  oc_sim* s = oc_create(&p);
  if (!s) return 4;
  oc_init(s, in, in + n, in + 2 * n, in + 3 * n, in + 5 * n);
  oc_step(s, steps);
  oc_fields(s, out, out + n, out + 2 * n, out + 3 * n, out + 5 * n, out + 7 * n, out + 8 * n);
  for (int i = 0; i < 9 * n; ++i)
    if (!isfinite(out[i])) {
      fprintf(stderr, "non-finite value at %d\n", i);
      return 5;
    }
  oc_destroy(s);
  free(in);
  free(out);
  printf("ok %dx%d %d steps n_sub %d\n", nx, ny, steps, n_sub);
  return 0;
}
