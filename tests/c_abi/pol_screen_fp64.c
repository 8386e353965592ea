/* Plain-C use of libgw: the FP64 polarization (Eq. polar_MB on the imaginary
 * axis) and the screening W = (1 - vP)^-1 v (Eq. W_Dyson) through the C ABI
 * on device buffers from hipMalloc, without Python.
 *
 * usage: pol_screen_fp64 <inputs.bin> <outputs.bin>
 * inputs (little-endian): int32 n_k, N, R, n_occ, n_unocc, n_omega; float64
 * omega[n_omega], eps[n_k][n_occ + n_unocc], v[N]; complex128 U[N][R],
 * psi[n_k][n_occ + n_unocc][R].  outputs: complex128 P[n_omega][N][N], then
 * W[n_omega][N][N].  Exit status 0 on success, 1 on a library or HIP error,
 * 2 on an I/O error, 3 if the screening reports a non-positive pivot. */
#include <hip/hip_runtime_api.h>
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
  int hdr[6];
  if (!f || fread(hdr, sizeof(int), 6, f) != 6) return 2;
  const int n_k = hdr[0], N = hdr[1], R = hdr[2], n_occ = hdr[3], n_unocc = hdr[4], n_omega = hdr[5];
  const int nb = n_occ + n_unocc;
  const size_t nU = (size_t)N * R * 16, nPsi = (size_t)n_k * nb * R * 16, nP = (size_t)n_omega * N * N * 16;
  double* omega = read_n(f, (size_t)n_omega * 8);
  double* eps = read_n(f, (size_t)n_k * nb * 8);
  double* v = read_n(f, (size_t)N * 8);
  void* U = read_n(f, nU);
  void* psi = read_n(f, nPsi);
  fclose(f);
  if (!omega || !eps || !v || !U || !psi) return 2;

  void *dU = to_device(U, nU), *dpsi = to_device(psi, nPsi), *deps = to_device(eps, (size_t)n_k * nb * 8);
  void* dv = to_device(v, (size_t)N * 8);
  void *dP = NULL, *dW = NULL, *dinfo = NULL, *ws = NULL, *ws2 = NULL;
  if (!dU || !dpsi || !deps || !dv) return 1;
  if (!hip_ok(hipMalloc(&dP, nP), "hipMalloc P") || !hip_ok(hipMalloc(&dW, nP), "hipMalloc W") ||
      !hip_ok(hipMalloc(&dinfo, (size_t)n_omega * sizeof(int)), "hipMalloc info"))
    return 1;

  gw_pol_desc d;
  memset(&d, 0, sizeof d);
  d.precision = GW_FP64;
  d.n_k = n_k;
  d.N = N;
  d.R = R;
  d.n_occ = n_occ;
  d.n_unocc = n_unocc;
  d.occ_begin = 0;
  d.occ_end = n_occ;
  d.unocc_begin = 0;
  d.unocc_end = n_unocc;
  d.n_omega = n_omega;
  d.omega_host = omega;
  d.kq_host = NULL; /* (k + 1) mod n_k */
  d.k_list_host = NULL;
  d.U = dU;
  d.psi = dpsi;
  d.eps = deps;
  d.eps_host = eps;
  d.P = dP;
  size_t bytes = 0, bytes2 = 0;
  if (!gw_ok(gw_polarization_workspace_size(&d, &bytes), "gw_polarization_workspace_size")) return 1;
  if (!gw_ok(gw_screen_workspace_size(N, n_omega, &bytes2), "gw_screen_workspace_size")) return 1;
  if (!hip_ok(hipMalloc(&ws, bytes ? bytes : 1), "hipMalloc ws") ||
      !hip_ok(hipMalloc(&ws2, bytes2 ? bytes2 : 1), "hipMalloc ws2"))
    return 1;
  if (!gw_ok(gw_polarization(NULL, &d, ws, bytes), "gw_polarization")) return 1;
  if (!gw_ok(gw_screen(NULL, N, n_omega, dP, dv, dW, dinfo, ws2, bytes2), "gw_screen")) return 1;
  if (!hip_ok(hipDeviceSynchronize(), "hipDeviceSynchronize")) return 1;

  void* P = malloc(nP);
  void* W = malloc(nP);
  int* info = malloc((size_t)n_omega * sizeof(int));
  if (!P || !W || !info) return 2;
  if (!hip_ok(hipMemcpy(P, dP, nP, hipMemcpyDeviceToHost), "hipMemcpy P") ||
      !hip_ok(hipMemcpy(W, dW, nP, hipMemcpyDeviceToHost), "hipMemcpy W") ||
      !hip_ok(hipMemcpy(info, dinfo, (size_t)n_omega * sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy info"))
    return 1;
  for (int j = 0; j < n_omega; ++j)
    if (info[j] != 0) {
      fprintf(stderr, "screening: frequency %d: info %d\n", j, info[j]);
      return 3;
    }
  FILE* o = fopen(argv[2], "wb");
  if (!o || fwrite(P, 1, nP, o) != nP || fwrite(W, 1, nP, o) != nP) return 2;
  fclose(o);
  hipFree(dU);
  hipFree(dpsi);
  hipFree(deps);
  hipFree(dv);
  hipFree(dP);
  hipFree(dW);
  hipFree(dinfo);
  hipFree(ws);
  hipFree(ws2);
  free(omega);
  free(eps);
  free(v);
  free(U);
  free(psi);
  free(P);
  free(W);
  free(info);
  printf("pol_screen_fp64: N=%d n_omega=%d ok\n", N, n_omega);
  return 0;
}
