/* A plain C host program that drives the library through include/rlb.h
 * alone: no Python and no torch. It sizes and allocates the workspace itself
 * (the library allocates nothing), creates a stream, initialises one lattice
 * from host fields, advances it, and writes the recovered fields and the
 * lattice sums back to a file. The GPU test compares that output with the
 * Python binding's run of the same lattice (bit for bit) and with the oracle.
 *
 * usage: rlb_run nx ny nz bcx bcy bcz tau_f tau_v tau_e tau_eps precision
 *                nsteps in.bin out.bin
 *   in.bin:  n0, eps0 (ncells doubles each), u0 (3 * ncells)
 *   out.bin: n, eps, P, gamma (ncells each), u (3 * ncells), sums (5),
 *            n_unphysical (one int64)
 * Exit status 0 on success; otherwise the failing call and its status are
 * printed and the status is 1 (2 for bad arguments or files). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "rlb.h"

static int fail(const char* what, int st) {
  fprintf(stderr, "rlb_run: %s failed: %d (%s)\n", what, st, rlb_status_string((rlb_status)st));
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 15) {
    fprintf(stderr, "usage: rlb_run nx ny nz bcx bcy bcz tau_f tau_v tau_e tau_eps "
                    "precision nsteps in.bin out.bin\n");
    return 2;
  }
  rlb_params p;
  memset(&p, 0, sizeof(p));
  p.nx = atoi(argv[1]);
  p.ny = atoi(argv[2]);
  p.nz = atoi(argv[3]);
  for (int k = 0; k < 3; ++k) p.bc[k] = atoi(argv[4 + k]);
  p.tau_f = atof(argv[7]);
  p.tau_v = atof(argv[8]);
  p.tau_e = atof(argv[9]);
  p.tau_eps = atof(argv[10]);
  rlb_options o;
  memset(&o, 0, sizeof(o));
  o.precision = atoi(argv[11]);
  const int32_t nsteps = atoi(argv[12]);
  if (p.nx < 1 || p.ny < 1 || p.nz < 1 || nsteps < 0) return 2;
  const size_t nc = (size_t)p.nx * p.ny * p.nz;

  double* in = (double*)malloc(5 * nc * sizeof(double));
  double* out = (double*)malloc(7 * nc * sizeof(double));
  if (!in || !out) return 2;
  FILE* fi = fopen(argv[13], "rb");
  if (!fi || fread(in, sizeof(double), 5 * nc, fi) != 5 * nc) {
    fprintf(stderr, "rlb_run: cannot read %s\n", argv[13]);
    return 2;
  }
  fclose(fi);

  size_t bytes = 0;
  int st = rlb_workspace_size(&p, 1, &o, &bytes);
  if (st != RLB_OK) return fail("rlb_workspace_size", st);
  void* ws = NULL;
  hipStream_t stream = NULL;
  if (hipMalloc(&ws, bytes) != hipSuccess) return fail("hipMalloc", RLB_E_DEVICE);
  if (hipStreamCreate(&stream) != hipSuccess) return fail("hipStreamCreate", RLB_E_DEVICE);

  rlb_handle h = NULL;
  st = rlb_init(&h, &p, 1, &o, in, in + nc, in + 2 * nc, 0, ws, bytes, (void*)stream);
  if (st != RLB_OK) return fail("rlb_init", st);
  st = rlb_step(h, nsteps);
  if (st != RLB_OK) return fail("rlb_step", st);
  double sums[5];
  int64_t bad = 0;
  st = rlb_moments(h, out, out + nc, out + 2 * nc, out + 3 * nc, out + 4 * nc, sums, &bad, 0);
  if (st != RLB_OK && st != RLB_E_UNPHYSICAL) return fail("rlb_moments", st);
  char kernel[128];
  int64_t steps = 0;
  st = rlb_info(h, &steps, kernel, sizeof(kernel));
  if (st != RLB_OK) return fail("rlb_info", st);
  rlb_free(h);
  (void)hipStreamDestroy(stream);
  (void)hipFree(ws);

  FILE* fo = fopen(argv[14], "wb");
  if (!fo || fwrite(out, sizeof(double), 7 * nc, fo) != 7 * nc ||
      fwrite(sums, sizeof(double), 5, fo) != 5 || fwrite(&bad, sizeof(bad), 1, fo) != 1) {
    fprintf(stderr, "rlb_run: cannot write %s\n", argv[14]);
    return 2;
  }
  fclose(fo);
  printf("rlb_run: %lld steps with %s, %lld inadmissible cell-updates\n", (long long)steps, kernel,
         (long long)bad);
  free(in);
  free(out);
  return 0;
}
