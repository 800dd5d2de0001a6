/* Runs the CPU oracle on the states and fields in a directory of raw
 * little-endian files (written by tests/test_sanitized_builds.py), so that the
 * oracle can be built with AddressSanitizer and UndefinedBehaviorSanitizer and
 * exercised outside Python. Test infrastructure only.
 *
 * usage: sanitize_driver DIR NX NY H DT STEPS
 * DIR holds c.u8 cc.u8 hoff.f64 voff.f64 u.f64 v.f64 in the library layout. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_step(int nx, int ny, double h, uint8_t *c, uint8_t *cc, double *hoff, double *voff, const double *u,
            const double *v, double dt, int64_t step, int flags, int64_t *st);
int or_fraction(int nx, int ny, const uint8_t *c, const uint8_t *cc, const double *hoff, const double *voff,
                double *C);
int or_curvature(int nx, int ny, double h, const uint8_t *c, const double *hoff, const double *voff, const double *C,
                 double *K, int64_t *st);
int or_ns_fields(int nx, int ny, double h, const uint8_t *c, const double *C, const double *K, double rho1,
                 double rho2, double mu1, double mu2, double sigma, double *rho, double *mu, double *fx, double *fy);
int or_counter_count(void);

static void *load(const char *dir, const char *name, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE *f = fopen(path, "rb");
  if (!f) { perror(path); exit(2); }
  void *p = malloc(bytes);
  if (!p || fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
  fclose(f);
  return p;
}

int main(int argc, char **argv) {
  if (argc != 7) return 2;
  const char *dir = argv[1];
  const int nx = atoi(argv[2]), ny = atoi(argv[3]), steps = atoi(argv[6]);
  const double h = atof(argv[4]), dt = atof(argv[5]);
  const size_t nn = (size_t)(nx + 1) * (ny + 1), nc = (size_t)nx * ny, nh = (size_t)nx * (ny + 1),
               nv = (size_t)(nx + 1) * ny;
  uint8_t *c = load(dir, "c.u8", nn), *cc = load(dir, "cc.u8", nc);
  double *hoff = load(dir, "hoff.f64", nh * 8), *voff = load(dir, "voff.f64", nv * 8);
  double *u = load(dir, "u.f64", nv * 8), *v = load(dir, "v.f64", nh * 8);
  int64_t *st = calloc((size_t)or_counter_count(), sizeof(int64_t));
  double *C = malloc(nc * 8), *K = malloc(nc * 8), *rho = malloc(nc * 8), *mu = malloc(nc * 8);
  double *fx = malloc(nv * 8), *fy = malloc(nh * 8);
  for (int k = 0; k < steps; k++) {
    for (int flags = 0; flags < 1; flags++) {
      const int rc = or_step(nx, ny, h, c, cc, hoff, voff, u, v, dt, k, flags, st);
      if (rc) { fprintf(stderr, "step %d rc %d\n", k, rc); return 3; }
    }
    or_fraction(nx, ny, c, cc, hoff, voff, C);
    or_curvature(nx, ny, h, c, hoff, voff, C, K, st);
    or_ns_fields(nx, ny, h, c, C, K, 1000.0, 1.0, 1e-3, 1e-5, 0.07, rho, mu, fx, fy);
  }
  printf("markers %lld ties %lld\n", (long long)st[0], (long long)st[3]);
  free(c); free(cc); free(hoff); free(voff); free(u); free(v); free(st);
  free(C); free(K); free(rho); free(mu); free(fx); free(fy);
  return 0;
}
