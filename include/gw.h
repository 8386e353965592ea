/*
 * gw.h -- C ABI of libgw: the RPA polarization matrix P_IJ(q, i w) in a
 * product basis and the screened interaction W on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method (Friedrich, Bluegel, Schindlmayr, all-electron GW in FLAPW):
 *   projections   M_I^{k n n'} = sum_r U[I][r] conj(psi_k[n][r]) psi_kq[n'][r]
 *                 (Sec. "Formulation in the MPB", Eq. proj_MB, on a grid; U
 *                 stands for the conjugated basis functions times the grid
 *                 quadrature weight)
 *   polarization  P_IJ(i w) = sum_k sum_{n occ} sum_{n' unocc}
 *                     w_{knn'}(w) M_I^{knn'} conj(M_J^{knn'}),
 *                 w = 4 D / (D^2 + w^2), D = eps_k[n] - eps_kq[n'] < 0
 *                 (Eq. polar_MB; its frequency bracket taken on the imaginary
 *                 axis, where it is real and P is Hermitian, summed over two
 *                 degenerate spins)
 *   screening     W = (1 - v P)^-1 v for the diagonal Coulomb eigenvalues v,
 *                 computed in the symmetrised form of Eqs. dielec_MB /
 *                 screen_MB: eps = 1 - sqrt(v) P sqrt(v), W = sqrt(v) eps^-1 sqrt(v)
 *
 * Conventions for every entry point:
 *  - Complex numbers are interleaved (re, im).  "c128" = two doubles, "c64" =
 *    two floats.  All matrices are row-major with the last index contiguous.
 *  - Pointers named *_host are host memory; every other pointer is device
 *    memory owned by the caller.  The library keeps no pointer after the call
 *    returns and allocates no device memory of its own: scratch space is the
 *    caller's workspace (size from the matching *_workspace_size query).
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued asynchronously on it; synchronise the stream before reading
 *    outputs.  Calls on different streams need different workspaces.
 *  - Every call validates its arguments on the host before enqueuing
 *    anything; on failure nothing is enqueued, the return value is a negative
 *    gw_status and gw_last_error() describes the problem.  No entry point
 *    aborts the process.
 *  - Results are deterministic: every output tile has one owner, no atomics.
 */
#ifndef GW_H
#define GW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic of the projection and accumulation steps.  The output P is
 * always c128; partial sums of at most one chunk of transition pairs are held
 * in the working precision and then added into P in FP64.
 *   GW_FP64        c128 inputs, FP64 arithmetic throughout.
 *   GW_FP32        c64 inputs, FP32 matrix-core (MFMA) arithmetic.
 *   GW_SPLIT_BF16  c64 inputs; every operand x is split into hi = bf16(x) and
 *                  lo = bf16(x - hi) (round to nearest even) and a product is
 *                  hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulation.
 *   GW_SPLIT_FP16  as SPLIT_BF16 with FP16 words; lo is pre-scaled by 2^11 and
 *                  accumulated separately so it stays in FP16's normal range. */
typedef enum gw_precision {
  GW_FP64 = 0,
  GW_FP32 = 1,
  GW_SPLIT_BF16 = 2,
  GW_SPLIT_FP16 = 3
} gw_precision;

typedef enum gw_status {
  GW_OK = 0,
  GW_ERR_INVALID_ARG = -1,  /* bad size, null pointer, non-insulating energies, w < 0 ... */
  GW_ERR_UNSUPPORTED = -2,  /* valid request the library does not implement */
  GW_ERR_WORKSPACE = -3,    /* workspace pointer null or smaller than required */
  GW_ERR_HIP = -4           /* a HIP runtime call failed (message has the HIP error) */
} gw_status;

/* Message for the last non-OK status returned on the calling thread. */
const char* gw_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int gw_version(void);

/* ------------------------------------------------------------------ projection
 * gw_project: M[I][n*n_unocc + n'] = sum_r U[I][r] conj(psi_occ[n][r]) psi_unocc[n'][r]
 * (Eq. proj_MB).
 *   precision  GW_FP64: U, psi_occ, psi_unocc, M are c128.
 *              GW_FP32 / GW_SPLIT_BF16 / GW_SPLIT_FP16: inputs c64, M c64.
 *   U          [N][R];  psi_occ [n_occ][R];  psi_unocc [n_unocc][R]
 *   M          [N][n_occ*n_unocc] (output, overwritten)
 *   N, R, n_occ, n_unocc >= 1.  ws/ws_bytes: workspace from
 *   gw_project_workspace_size (may be NULL/0 when the size is 0). */
int gw_project_workspace_size(int precision, int N, int R, int n_occ, int n_unocc,
                              size_t* bytes_host);
int gw_project(void* stream, int precision, int N, int R, int n_occ, int n_unocc,
               const void* U, const void* psi_occ, const void* psi_unocc, void* M,
               void* ws, size_t ws_bytes);

/* ---------------------------------------------------------------- polarization
 * gw_polarization: P(i w_j) for one response momentum q (Eq. polar_MB on the
 * imaginary axis), summed over the k-points in k_list_host with the occupied
 * bands of set k and the unoccupied bands of set kq[k].
 *
 * Band layout of each k-set: bands [0, n_occ) are occupied, bands
 * [n_occ, n_occ + n_unocc) unoccupied; psi and eps use that order.  The sum
 * runs over occupied bands [occ_begin, occ_end) and unoccupied bands
 * [n_occ + unocc_begin, n_occ + unocc_end), so a truncated band sum (bands up
 * to a cutoff) and sampled subsets are plain sub-ranges; P is additive over
 * disjoint ranges and k subsets (use accumulate = 1).
 *
 * Every pair summed must have eps_k[n] < eps_kq[n'] (insulator); otherwise
 * GW_ERR_INVALID_ARG.  omega_host entries must be finite and >= 0.
 * P is the full Hermitian matrix; its diagonal is stored with zero imaginary
 * part. */
typedef struct gw_pol_desc {
  int precision;            /* gw_precision */
  int n_k;                  /* k-sets held in psi / eps */
  int N;                    /* basis size (rows of U) */
  int R;                    /* grid points */
  int n_occ, n_unocc;       /* band split of every k-set */
  int occ_begin, occ_end;   /* occupied bands summed, 0 <= begin < end <= n_occ */
  int unocc_begin, unocc_end; /* unoccupied bands summed, 0 <= begin < end <= n_unocc */
  int n_omega;              /* >= 1 */
  const double* omega_host; /* [n_omega] imaginary frequencies (Hartree), >= 0 */
  const int* kq_host;       /* [n_k] k+q set of each k; NULL means (k+1) mod n_k */
  const int* k_list_host;   /* [n_k_list] k-points summed; NULL means all n_k */
  int n_k_list;
  const void* U;            /* [N][R] c128 (FP64) or c64 (other precisions) */
  const void* psi;          /* [n_k][n_occ+n_unocc][R] same dtype as U */
  const double* eps;        /* [n_k][n_occ+n_unocc] band energies (device) */
  const double* eps_host;   /* the same values in host memory (validation) */
  double* P;                /* [n_omega][N][N] c128 output */
  int accumulate;           /* 0: P is overwritten; 1: the sum is added to P */
  int chunk_pairs;          /* transition pairs per chunk; 0 = library default */
} gw_pol_desc;

int gw_polarization_workspace_size(const gw_pol_desc* desc_host, size_t* bytes_host);
int gw_polarization(void* stream, const gw_pol_desc* desc_host, void* ws, size_t ws_bytes);

/* ------------------------------------------------------------------ screening
 * gw_screen: W(i w_j) = (1 - diag(v) P_j)^-1 diag(v) for j < n_omega (Eq.
 * W_Dyson in matrix form), computed as sqrt(v) eps^-1 sqrt(v) with the
 * Hermitian eps = 1 - sqrt(v) P sqrt(v) (Eqs. dielec_MB, screen_MB) inverted
 * in FP64 by a blocked Gauss-Jordan sweep without pivoting, which is stable
 * for Hermitian positive definite eps (eps >= 1 whenever P <= 0).
 *   P       [n_omega][N][N] c128, Hermitian (only the lower triangle is read)
 *   v       [N] doubles > 0
 *   W       [n_omega][N][N] c128 output (full Hermitian matrix); may not alias P
 *   info    [n_omega] ints (device), written: 0 on success, c+1 if the pivot
 *           block starting at column c was not positive definite (W_j is then
 *           undefined).  Read it after synchronising the stream. */
int gw_screen_workspace_size(int N, int n_omega, size_t* bytes_host);
int gw_screen(void* stream, int N, int n_omega, const double* P, const double* v, double* W,
              int* info, void* ws, size_t ws_bytes);


/* ------------------------------------------------------------------ profiling
 * Optional per-kernel timing with HIP events recorded on the caller's stream
 * around every launch of the library's main kernels (projection,
 * accumulation, screening update, ...).  Off by default.
 *   gw_profile_enable(1) starts recording, gw_profile_enable(0) stops.
 *   gw_profile_reset() drops all records.
 *   gw_profile_query(name, &launches, &total_ms) synchronises the recorded
 *   events and sums the durations of the launches of kernel `name` (the
 *   kernel's function name, e.g. "project_bf16_kernel"); unknown names give
 *   launches = 0.  Host-side bookkeeping only; safe to call from one thread. */
int gw_profile_enable(int on);
int gw_profile_reset(void);
int gw_profile_query(const char* kernel_name_host, int* launches_host, double* total_ms_host);

#ifdef __cplusplus
}
#endif
#endif /* GW_H */
