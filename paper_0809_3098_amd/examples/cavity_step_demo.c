/*
 * A plain C caller of the library: no Python, no torch.  Creates one cavity
 * in a workspace from hipMalloc, advances it, and writes psi then omega
 * (n*n doubles each, row-major [j][i]) to a file, with the last step's
 * monitors on stdout.
 *
 * usage: cavity_step_demo N RE STEPS OUT_FILE
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "cavity.h"

static int hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s failed: %s\n", what, hipGetErrorString(e));
    return 0;
  }
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: %s N RE STEPS OUT_FILE\n", argv[0]);
    return 2;
  }
  cavity_params p;
  memset(&p, 0, sizeof p); /* zero selects every default */
  p.n = atoi(argv[1]);
  p.re = atof(argv[2]);
  p.u_lid = 1.0;
  const int steps = atoi(argv[3]);
  size_t bytes = 0;
  if (cavity_workspace_bytes(&p, 1, &bytes) != CAVITY_OK) {
    fprintf(stderr, "%s\n", cavity_last_error());
    return 1;
  }
  void* ws = NULL;
  double* d_out = NULL;
  const size_t field = (size_t)p.n * p.n * sizeof(double);
  if (!hip_ok(hipMalloc(&ws, bytes), "hipMalloc") ||
      !hip_ok(hipMalloc((void**)&d_out, 2 * field), "hipMalloc"))
    return 1;
  cavity_t h = NULL;
  cavity_stats st;
  int rc = cavity_create(&p, 1, ws, bytes, NULL, &h);
  if (rc == CAVITY_OK) rc = cavity_step(h, steps, &st);
  if (rc == CAVITY_OK) rc = cavity_fields(h, 0, d_out, d_out + (size_t)p.n * p.n, NULL, NULL);
  if (rc != CAVITY_OK) {
    fprintf(stderr, "status %d: %s\n", rc, cavity_last_error());
    return 1;
  }
  double* host = (double*)malloc(2 * field);
  if (!host || !hip_ok(hipDeviceSynchronize(), "hipDeviceSynchronize") ||
      !hip_ok(hipMemcpy(host, d_out, 2 * field, hipMemcpyDeviceToHost), "hipMemcpy"))
    return 1;
  FILE* f = fopen(argv[4], "wb");
  if (!f || fwrite(host, 1, 2 * field, f) != 2 * field) {
    fprintf(stderr, "cannot write %s\n", argv[4]);
    return 1;
  }
  fclose(f);
  printf("step %lld res_psi %.17g res_omega %.17g ke %.17g sweeps %lld\n", (long long)st.step,
         st.res_psi, st.res_omega, st.ke, (long long)st.sweeps_total);
  cavity_destroy(h);
  free(host);
  hipFree(d_out);
  hipFree(ws);
  return 0;
}
