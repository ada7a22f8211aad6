/*
 * Host-only use of the C-ABI from C: describes the 2x2x2-patch unit cube
 * (p = 2, 4 elements per row, conductors below z = 0.5, the curl-form source
 * sin^2(pi x) sin^2(pi y) in the insulators), creates the handle (host work
 * only, no GPU), and prints the topology counts and device footprints.  The
 * test that builds it compares the output with the Python binding.
 */
#include <math.h>
#include <stdio.h>

#include "tcf.h"

static void phi(const double* xs, int32_t nx, const double* ys, int32_t ny, const double* zs,
                int32_t nz, int32_t k, double* out, void* ctx) {
  (void)zs; (void)k; (void)ctx;
  const double pi = 3.14159265358979323846;
  for (int iz = 0; iz < nz; ++iz)
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nx; ++ix) {
        const double sx = sin(pi * xs[ix]), sy = sin(pi * ys[iy]);
        out[ix + nx * (iy + ny * iz)] = sx * sx * sy * sy;
      }
}

int main(void) {
  const double br[3] = {0.0, 0.5, 1.0};
  const int32_t nel[2] = {4, 4}, deg[2] = {2, 2};
  double sigma[8], nu[8], amp[20];
  uint8_t src[8];
  for (int s = 0; s < 8; ++s) {
    const int k = s / 4;
    sigma[s] = k == 0 ? 1e6 : 0.0;
    nu[s] = 1.0 / (4e-7 * 3.14159265358979323846);
    src[s] = sigma[s] == 0.0;
  }
  for (int l = 0; l < 20; ++l) amp[l] = sin(2 * 3.14159265358979323846 * 50 * 1e-4 * (l + 1));
  tcf_problem_desc d = {0};
  for (int a = 0; a < 3; ++a) {
    d.np[a] = 2;
    d.breaks[a] = br;
    d.nel[a] = nel;
    d.deg[a] = deg;
  }
  d.sigma = sigma;
  d.nu = nu;
  d.src_mask = src;
  d.n_rhs = 1;
  d.phi = phi;
  d.amp = amp;
  d.dt = 1e-4;
  d.n_steps = 20;
  tcf_options o;
  tcf_default_options(&o);
  tcf_problem* h = NULL;
  int rc = tcf_create(&d, &o, NULL, &h);
  if (rc != TCF_OK) {
    printf("create failed %d: %s\n", rc, tcf_last_error(NULL));
    return 1;
  }
  int64_t cnt[16];
  size_t len = 16;
  rc = tcf_get_topology(h, TCF_TOPO_COUNTS, cnt, &len);
  if (rc != TCF_OK) return 2;
  printf("counts");
  for (size_t i = 0; i < len; ++i) printf(" %lld", (long long)cnt[i]);
  printf("\n");
  size_t b64 = 0, b32 = 0;
  if (tcf_footprint(h, &b64, &b32) != TCF_OK) return 3;
  printf("footprint %zu %zu\n", b64, b32);
  /* a step before setup is a call-order error */
  printf("step_before_setup %d\n", tcf_step(h, 1, NULL));
  /* an invalid description is rejected with a message */
  sigma[3] = -1.0;
  tcf_problem* bad = NULL;
  rc = tcf_create(&d, &o, NULL, &bad);
  printf("negative_sigma %d %s\n", rc, bad == NULL ? "null" : "handle");
  tcf_destroy(h);
  return 0;
}
