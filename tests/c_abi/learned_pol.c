/* Plain-C use of the learned path of libgw: P over all bands with the
 * unoccupied bands above a cutoff replaced by the perceptron's correction,
 * judged against an explicit sample (gw_polarization_learned), on device
 * buffers from hipMalloc, without Python.
 *
 * usage: learned_pol <inputs.bin> <outputs.bin>
 * inputs (little-endian): int32 precision, n_k, N, R, n_occ, n_unocc, n_omega,
 * cut, n_sample_occ, n_in, width, n_out; float64 judge_tol, omega[n_omega],
 * eps[n_k][n_occ + n_unocc]; U[N][R] and psi[n_k][n_occ + n_unocc][R]
 * (complex128 for GW_FP64, complex64 otherwise); float32 master[n_params]
 * (perceptron parameters in the layout of gw.h).  outputs: complex128
 * P[n_omega][N][N], float64 err[n_omega], int32 used_fallback.  Exit status 0
 * on success, 1 on a library or HIP error, 2 on an I/O error. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gw.h"

static int hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 0;
  }
  return 1;
}

static int gw_ok(int st, const char* what) {
  if (st != GW_OK) {
    fprintf(stderr, "%s: status %d: %s\n", what, st, gw_last_error());
    return 0;
  }
  return 1;
}

static void* read_n(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (p && fread(p, 1, bytes, f) != bytes) {
    free(p);
    return NULL;
  }
  return p;
}

static void* to_device(const void* h, size_t bytes) {
  void* d = NULL;
  if (!hip_ok(hipMalloc(&d, bytes), "hipMalloc")) return NULL;
  if (!hip_ok(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice), "hipMemcpy to device")) return NULL;
  return d;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s inputs.bin outputs.bin\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  int h[12];
  double tol = 0.0;
  if (!f || fread(h, sizeof(int), 12, f) != 12 || fread(&tol, sizeof(double), 1, f) != 1) return 2;
  const int prec = h[0], n_k = h[1], N = h[2], R = h[3], n_occ = h[4], n_unocc = h[5], n_omega = h[6];
  const int cut = h[7], n_sample = h[8], n_in = h[9], width = h[10], n_out = h[11];
  const int nb = n_occ + n_unocc;
  const size_t cb = prec == GW_FP64 ? 16 : 8;
  const size_t nU = (size_t)N * R * cb, nPsi = (size_t)n_k * nb * R * cb, nP = (size_t)n_omega * N * N * 16;
  size_t n_params = 0, n_bf16 = 0;
  if (!gw_ok(gw_mlp_sizes(n_in, width, n_out, &n_params, &n_bf16), "gw_mlp_sizes")) return 1;
  double* omega = read_n(f, (size_t)n_omega * 8);
  double* eps = read_n(f, (size_t)n_k * nb * 8);
  void* U = read_n(f, nU);
  void* psi = read_n(f, nPsi);
  float* master = read_n(f, n_params * sizeof(float));
  fclose(f);
  if (!omega || !eps || !U || !psi || !master) return 2;

  void *dU = to_device(U, nU), *dpsi = to_device(psi, nPsi), *deps = to_device(eps, (size_t)n_k * nb * 8);
  void* dmaster = to_device(master, n_params * sizeof(float));
  void *dP = NULL, *dwt = NULL, *dwk = NULL, *ws = NULL;
  if (!dU || !dpsi || !deps || !dmaster) return 1;
  if (!hip_ok(hipMalloc(&dP, nP), "hipMalloc P") || !hip_ok(hipMalloc(&dwt, n_bf16 * 2), "hipMalloc wt") ||
      !hip_ok(hipMalloc(&dwk, n_bf16 * 2), "hipMalloc wk"))
    return 1;

  gw_mlp m;
  memset(&m, 0, sizeof m);
  m.n_in = n_in;
  m.width = width;
  m.n_out = n_out;
  m.master = (float*)dmaster;
  m.wt = (uint16_t*)dwt;
  m.wk = (uint16_t*)dwk;
  if (!gw_ok(gw_mlp_sync_bf16(NULL, &m), "gw_mlp_sync_bf16")) return 1;

  gw_pol_desc d;
  memset(&d, 0, sizeof d);
  d.precision = prec;
  d.n_k = n_k;
  d.N = N;
  d.R = R;
  d.n_occ = n_occ;
  d.n_unocc = n_unocc;
  d.occ_end = n_occ;
  d.unocc_end = n_unocc;
  d.n_omega = n_omega;
  d.omega_host = omega;
  d.U = dU;
  d.psi = dpsi;
  d.eps = deps;
  d.eps_host = eps;
  d.P = dP;

  double* err = calloc((size_t)n_omega, sizeof(double));
  int used_fallback = -1;
  gw_learned_desc l;
  memset(&l, 0, sizeof l);
  l.mlp = &m;
  l.cut = cut;
  l.judge = 1;
  l.n_sample_occ = n_sample;
  l.judge_tol = tol;
  l.judge_err_host = err;
  l.used_fallback_host = &used_fallback;

  size_t bytes = 0;
  if (!gw_ok(gw_polarization_learned_workspace_size(&d, &l, &bytes), "gw_polarization_learned_workspace_size"))
    return 1;
  if (!hip_ok(hipMalloc(&ws, bytes), "hipMalloc ws")) return 1;
  if (!gw_ok(gw_polarization_learned(NULL, &d, &l, ws, bytes), "gw_polarization_learned")) return 1;
  if (!hip_ok(hipDeviceSynchronize(), "hipDeviceSynchronize")) return 1;

  void* P = malloc(nP);
  if (!P || !err) return 2;
  if (!hip_ok(hipMemcpy(P, dP, nP, hipMemcpyDeviceToHost), "hipMemcpy P")) return 1;
  FILE* o = fopen(argv[2], "wb");
  if (!o || fwrite(P, 1, nP, o) != nP || fwrite(err, sizeof(double), (size_t)n_omega, o) != (size_t)n_omega ||
      fwrite(&used_fallback, sizeof(int), 1, o) != 1)
    return 2;
  fclose(o);
  hipFree(dU);
  hipFree(dpsi);
  hipFree(deps);
  hipFree(dmaster);
  hipFree(dP);
  hipFree(dwt);
  hipFree(dwk);
  hipFree(ws);
  free(omega);
  free(eps);
  free(U);
  free(psi);
  free(master);
  free(P);
  free(err);
  printf("learned_pol: N=%d n_omega=%d cut=%d fallback=%d ok\n", N, n_omega, cut, used_fallback);
  return 0;
}
