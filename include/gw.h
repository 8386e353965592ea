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
 *                  accumulated separately so it stays in FP16's normal range.
 *   GW_FP16        ablation: single FP16 products (the hi words of
 *                  GW_SPLIT_FP16, same power-of-two scaling, no lo words);
 *                  about 3e-4 relative error, above the 1e-4 bar of the
 *                  reduced-precision paths. */
typedef enum gw_precision {
  GW_FP64 = 0,
  GW_FP32 = 1,
  GW_SPLIT_BF16 = 2,
  GW_SPLIT_FP16 = 3,
  GW_FP16 = 4
} gw_precision;

typedef enum gw_status {
  GW_OK = 0,
  GW_ERR_INVALID_ARG = -1,  /* bad size, null pointer, non-insulating energies, w < 0 ... */
  GW_ERR_UNSUPPORTED = -2,  /* valid request the library does not implement */
  GW_ERR_WORKSPACE = -3,    /* workspace pointer null or smaller than required */
  GW_ERR_HIP = -4,          /* a HIP runtime call failed (message has the HIP error) */
  GW_ERR_NONFINITE = -5,    /* GW_CHECK_FINITE: an input or a result holds Inf or NaN */
  GW_ERR_NOT_HPD = -6       /* GW_CHECK_HPD: eps = 1 - sqrt(v) P sqrt(v) is not positive definite at some
                               frequency (P is not negative semidefinite, Eqs. dielec_MB / screen_MB) */
} gw_status;

/* Optional checks (gw_pol_desc.flags, gw_screen_ex).  Each makes the call
 * synchronise its stream, so a call with a check cannot be captured into a
 * graph.
 *   GW_CHECK_FINITE  the device inputs are scanned for Inf/NaN before any
 *                    other work (nothing else is enqueued when one is found)
 *                    and the results after the work; GW_ERR_NONFINITE names
 *                    which.
 *   GW_CHECK_HPD     gw_screen_ex: after the sweep, GW_ERR_NOT_HPD when a
 *                    frequency's eps met a non-positive pivot (info still
 *                    holds the failing column of every frequency). */
enum { GW_CHECK_FINITE = 1, GW_CHECK_HPD = 2 };

/* Message for the last non-OK status returned on the calling thread. */
const char* gw_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int gw_version(void);

/* ------------------------------------------------------------------ projection
 * gw_project: M[I][n*n_unocc + n'] = sum_r U[I][r] conj(psi_occ[n][r]) psi_unocc[n'][r]
 * (Eq. proj_MB).
 *   precision  GW_FP64: U, psi_occ, psi_unocc, M are c128.
 *              GW_FP32 / GW_SPLIT_BF16 / GW_SPLIT_FP16 / GW_FP16: inputs c64, M c64.
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
 * part.
 *
 * real_inputs = 1 (GW_SPLIT_BF16 only, else GW_ERR_UNSUPPORTED): U and psi
 * are real float32 arrays of the same shapes -- the inversion-symmetric case,
 * where a symmetrized basis makes the matrices real symmetric (Sec. "Mixed
 * product basis", Eq. condition_inv; the text after Eq. polar_MB).  Every product and P are then real; P is returned as c128 with zero
 * imaginary parts, and the contractions need a quarter of the MFMA work.
 *
 * n_nodes > 0 selects the spectral route of the text after Eq. polar_MB: the
 * spectral function (the imaginary part of P on the real axis, a delta
 * function at every transition energy x = eps_kq[n'] - eps_k[n]) is
 * accumulated on the transition-energy nodes nodes_host[0..n_nodes), each
 * transition's weight split linearly between the two nodes around x, and
 * P(i w_j) is the Hilbert transform of the node weights:
 *   P(i w_j) = sum_b -4 x_b / (x_b^2 + w_j^2) sum_t h_b(x_t) M_t M_t^H.
 * It is exact when every transition sits on a node and otherwise interpolates
 * the bracket linearly in x between nodes (error falling as the square of the
 * node spacing).  2 <= n_nodes <= 256 (<= 64 with GW_SPLIT_FP16), nodes
 * finite, > 0 and increasing, and every summed transition energy inside
 * [nodes[0], nodes[n_nodes-1]], else GW_ERR_INVALID_ARG (GW_ERR_UNSUPPORTED
 * for the node count with GW_SPLIT_FP16).  The workspace then also holds the
 * n_nodes node matrices (n_nodes * N * N * 16 bytes). */
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
  int real_inputs;          /* 1: U and psi are real float32 (see above); 0: complex */
  int n_nodes;              /* > 0: spectral route on these nodes (see above); 0: direct sum */
  const double* nodes_host; /* [n_nodes] transition-energy nodes (Hartree), increasing */
  int flags;                /* 0 or GW_CHECK_FINITE (U, psi, eps before; P after) */
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
 *   info    [n_omega] ints (device), written: 0 on success, c+1 if the
 *           elimination met a non-positive (or non-finite) pivot at column c,
 *           i.e. eps_j is not positive definite (W_j is then undefined).  Read
 *           it after synchronising the stream. */
int gw_screen_workspace_size(int N, int n_omega, size_t* bytes_host);
int gw_screen(void* stream, int N, int n_omega, const double* P, const double* v, double* W,
              int* info, void* ws, size_t ws_bytes);
/* gw_screen with checks: flags is 0 or a combination of GW_CHECK_FINITE (P
 * and v before the sweep, W after it) and GW_CHECK_HPD (see above).  With
 * flags = 0 it is gw_screen. */
int gw_screen_ex(void* stream, int N, int n_omega, const double* P, const double* v, double* W, int* info,
                 int flags, void* ws, size_t ws_bytes);

/* gw_screen_noalloc: gw_screen without a workspace, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  The sweep's panels live in a fixed
 * array of gw_screen_noalloc_max_bytes() bytes (64 MiB) that the library holds
 * on every GPU it runs on until the process ends; the call itself allocates
 * nothing.  Arguments, results and info as for gw_screen.  A size whose
 * panels exceed the array (gw_screen_workspace_size(N, n_omega) > the
 * maximum, e.g. N > ~4000 at 16 frequencies) gives GW_ERR_WORKSPACE with
 * nothing enqueued.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or threads without ordering) race and
 * must be serialised by the caller.  Each call writes every panel element it
 * reads, so no clearing is needed between calls. */
size_t gw_screen_noalloc_max_bytes(void);
int gw_screen_noalloc(void* stream, int N, int n_omega, const double* P, const double* v, double* W, int* info);


/* ----------------------------------------------------------- learned high-band part
 * The unoccupied bands above a cutoff are left out of the explicit sum and
 * their contribution to P is predicted by a small perceptron (the paper's
 * extrapolar correction, text after Eq. SEc_AC / Fig. nband, targets the same
 * truncation with a fixed-energy completeness argument; here the correction is
 * learned from full-band runs).
 *
 * Perceptron: h1 = silu(x W1 + b1), h2 = silu(h1 W2 + b2), y = h2 W3 + b3,
 * silu(z) = z sigmoid(z).  Parameters live in caller-owned device buffers:
 *   master  FP32 [W1 n_in*width][b1 width][W2 width*width][b2 width]
 *                [W3 width*n_out][b3 n_out], each W row-major [in][out]
 *   adam_m, adam_v  FP32, same layout (needed by gw_mlp_adam_step only)
 *   wt      BF16 copies of W1, W2, W3 transposed ([out][in]), concatenated
 *   wk      BF16 copies of W1, W2, W3 in master layout ([in][out])
 * n_in, width, n_out are each 32, 64, 128 or 256.  Matrix products use the
 * BF16 weights with FP32 accumulation; FP32 activations and gradients enter
 * as hi + lo BF16 pairs.  Row-major FP32 buffers must be 16-byte aligned. */
typedef struct gw_mlp {
  int n_in, width, n_out;
  float* master;
  float* adam_m;
  float* adam_v;
  uint16_t* wt;
  uint16_t* wk;
} gw_mlp;

/* Element counts of master (and of adam_m/adam_v) and of wt (= of wk). */
int gw_mlp_sizes(int n_in, int width, int n_out, size_t* n_params_host, size_t* n_bf16_host);
/* Refresh wt and wk from master (after loading or editing master). */
int gw_mlp_sync_bf16(void* stream, const gw_mlp* m_host);
/* Y [rows][n_out] from X [rows][n_in]; act (4*rows*width floats) receives
 * the blocks z1, h1, z2, h2, each [rows][width], for gw_mlp_backward. */
int gw_mlp_forward(void* stream, const gw_mlp* m_host, const float* X, int rows, float* Y, float* act);
/* loss[0] = (1/rows) sum 0.5 mask (Y - T)^2 over the first n_used columns of
 * Y [rows][n_out]; T and mask are [rows][n_used] (mask may be NULL);
 * dY [rows][n_out] = mask (Y - T) / rows (zero in unused columns). */
int gw_mlp_loss(void* stream, int rows, int n_out, int n_used, const float* Y, const float* T, const float* mask,
                float* dY, float* loss);
int gw_mlp_workspace_size(int rows, int width, size_t* bytes_host);
/* grad (master layout) = d loss / d params for the loss whose dY is given;
 * dX [rows][n_in] optional (NULL to skip).  act from gw_mlp_forward. */
int gw_mlp_backward(void* stream, const gw_mlp* m_host, const float* X, const float* act, const float* dY, int rows,
                    float* grad, float* dX, void* ws, size_t ws_bytes);
/* One Adam step (Kingma & Ba, bias-corrected, step counts from 1) on master;
 * refreshes wt and wk. */
int gw_mlp_adam_step(void* stream, const gw_mlp* m_host, const float* grad, float lr, float beta1, float beta2,
                     float eps, int step);

/* Inputs of the feature, judge and correction kernels.  P_ret is the explicit
 * sum over unoccupied bands [0, cut) (from gw_polarization). */
typedef struct gw_surr_desc {
  int N, n_omega;
  const double* omega_host;  /* [n_omega]; the first entry is the reference frequency */
  int n_k, n_occ, n_unocc;   /* band layout as in gw_pol_desc */
  int cut;                   /* explicit unoccupied bands, 1 <= cut <= n_unocc */
  const int* kq_host;        /* NULL means (k+1) mod n_k; n_k <= 64 */
  const double* eps;         /* device [n_k][n_occ+n_unocc] */
  const double* P_ret;       /* device [n_omega][N][N] c128 */
  int n_in;                  /* feature row length (multiple of 32, >= 12) */
} gw_surr_desc;

int gw_surrogate_workspace_size(const gw_surr_desc* d_host, size_t* bytes_host);
/* X [n_omega*N][n_in], row r = j*N + I: 12 features of basis function I at
 * frequency j (omega map, log of the left-out/retained weight sums of the
 * band energies, log profile and relative size of |P_ret,II|, I/N, band-edge
 * energies, retained fraction), zero padded. */
int gw_surrogate_features(void* stream, const gw_surr_desc* d_host, float* X, void* ws, size_t ws_bytes);
/* Training targets: T[r] = log((P_ret,II - P_full,II) / |P_ret,II|), mask 0
 * where undefined.  T and mask are [n_omega*N]. */
int gw_surrogate_targets(void* stream, int N, int n_omega, const double* P_ret, const double* P_full, float* T,
                         float* mask);
/* P_j[I][J] *= 1 + exp((y_jI + y_jJ)/2) with y_jI = Y[(j*N + I)*ldy]
 * (y clamped to [-30, 30]): P + D P D, D = diag(exp(y/2)). */
int gw_surrogate_apply(void* stream, int N, int n_omega, const float* Y, int ldy, double* P);
/* err[j] (device, n_omega doubles) = |TRs_j / f_j - TRp_j| / TRp_j with TRp
 * the predicted left-out trace, TRs the trace of P_sample (the explicit sum of
 * the left-out bands [cut, n_unocc) for the sample rows (k, occupied band)
 * given) and f_j the sample's share of the left-out weight sum. */
int gw_surrogate_judge(void* stream, const gw_surr_desc* d_host, const float* Y, int ldy, const double* P_sample,
                       int n_sample, const int* sample_k_host, const int* sample_occ_host, double* err, void* ws,
                       size_t ws_bytes);

/* ------------------------------------------------ learned path in one call
 * gw_polarization_learned: P(i w_j) over all bands with the unoccupied bands
 * above a cutoff replaced by the learned correction (the truncation that the
 * paper's extrapolar approximation targets, Sec. "Test calculations",
 * convergence with the number of bands), judged against an explicit sample
 * and, when the judge fails, replaced by the explicit sum:
 *   1. P_ret = gw_polarization over unoccupied bands [0, cut)
 *   2. X = gw_surrogate_features(P_ret), Y = gw_mlp_forward(X)
 *   3. judge (judge = 1): for n_sample_occ occupied bands of every k-set,
 *      spread evenly from the lowest to the highest (the middle one when
 *      n_sample_occ = 1), the left-out bands [cut, n_unocc) are projected
 *      (Eq. proj_MB) and their exact left-out trace sum_t |w_t| |M_t|^2 taken;
 *      err_j = |TR_sample,j / f_j - TR_pred,j| / TR_pred,j as for
 *      gw_surrogate_judge.  err is copied to the host (the one stream
 *      synchronisation of the call).
 *   4. if every err_j <= judge_tol: P = P_ret + D P_ret D (gw_surrogate_apply)
 *      else (fallback): the explicit sum over [cut, n_unocc) is added, so P is
 *      the all-band result of gw_polarization.
 * desc: as for gw_polarization over all bands: occ [0, n_occ), unocc [0,
 * n_unocc), k_list_host NULL, accumulate 0, n_nodes 0, real_inputs 0,
 * n_k <= 64; flags as there.  P is overwritten.  judge = 0 skips step 3 and
 * always applies the correction; the call is then asynchronous.
 * Workspace from gw_polarization_learned_workspace_size (the polarization
 * passes', the perceptron's activations and the judge's projections). */
typedef struct gw_learned_desc {
  const gw_mlp* mlp;        /* trained perceptron (host struct of device pointers; inference reads wt) */
  int cut;                  /* unoccupied bands summed explicitly, 1 <= cut < n_unocc */
  int judge;                /* 1: judge and fall back; 0: apply without judging */
  int n_sample_occ;         /* judge sample per k-set, 1 <= n_sample_occ <= n_occ, n_k * n_sample_occ <= 64 */
  double judge_tol;         /* largest accepted err_j (finite, >= 0) */
  double* judge_err_host;   /* optional host [n_omega] output: err_j (judge = 1) */
  int* used_fallback_host;  /* optional host output: 1 when the explicit sum replaced the correction */
} gw_learned_desc;

int gw_polarization_learned_workspace_size(const gw_pol_desc* desc_host, const gw_learned_desc* learned_host,
                                           size_t* bytes_host);
int gw_polarization_learned(void* stream, const gw_pol_desc* desc_host, const gw_learned_desc* learned_host,
                            void* ws, size_t ws_bytes);

/* ------------------------------------------------ basis optimization (v_min)
 * Sec. "Optimization of the MPB": only the Coulomb eigenfunctions with
 * eigenvalue v_mu >= v_min are kept (v_min = 0 restores the full basis).  With
 * the basis in the Coulomb eigenbasis (diagonal v) this compacts the rows of U
 * and the entries of v, preserving their order; the reduced U and v are then
 * passed to gw_polarization / gw_screen / gw_sigma_c unchanged.
 *
 * gw_basis_select_count: host-only; n_keep_host = #{i : v_host[i] >= v_min}.
 * gw_basis_select: U [N][R] device rows of elem_bytes-byte elements (4 real
 * float, 8 c64, 16 c128), v [N] device; writes U_out [n_keep][R], v_out
 * [n_keep] and src_of_dst [n_keep] (device: original row of each kept row).
 * n_keep must be the count above (the device recomputes the selection from
 * v, which must hold the same values as v_host); with n_keep = 0 nothing is
 * written and the output pointers may be NULL.  Asynchronous on stream. */
int gw_basis_select_count(int N, const double* v_host, double v_min, int* n_keep_host);
int gw_basis_select(void* stream, int N, int R, int elem_bytes, const void* U, const double* v, double v_min,
                    int n_keep, void* U_out, double* v_out, int* src_of_dst);

/* ------------------------------------------------- correlation self-energy
 * Diagonal correlation self-energy on the imaginary axis, Eq. SEc_AC (the
 * analytic continuation of Eq. SEc_MB), for a list of states (set s, band n):
 *
 *   sigma[i][o] = -(1/2pi) sum_t sum_n' sum_{mu,nu} conj(m_mu) Wc_{mu nu}(t) m_nu  (integrated)
 *               = -(1/2pi) sum_t sum_n'  int dw' q_{t n'}(i w') / (i w_o + i w' - (e_n' - mu))
 *
 * with m_I = sum_r U_Ir conj(psi_{s,n}(r)) psi_{s',n'}(r) (Eq. proj_MB), s' =
 * (s + t) mod n_k, n' over all n_bands bands of set s', Wc(t) = W(t) - diag(v),
 * and q_{t n'}(i w') = m^H Wc(t, i w') m between the mesh points interpolated
 * by a cubic spline in lambda = w/(1+w) (text after Eq. SEc_AC; zero slope at
 * w = 0, at the last point the slope of the w^-2 tail q_L (w_L/w)^2 used
 * beyond it), integrated in closed form.  W is even in w (P depends on w^2),
 * so the integral over w' < 0 is folded onto w' > 0.  No Gamma-point terms.
 *
 *   precision       GW_FP64 (U, psi c128) or GW_SPLIT_BF16 (U, psi c64; the
 *                   quadratic forms on the split-BF16 matrix cores)
 *   mesh_host       n_mesh (2..64) imaginary frequencies of W, mesh[0] = 0,
 *                   strictly increasing
 *   omega_out_host  n_out (1..64) frequencies >= 0 at which sigma is returned
 *   state_*_host    n_states states (set in [0,n_k), band in [0,n_bands))
 *   mu              chemical potential; every e - mu must be nonzero
 *   U, psi, eps     as for gw_polarization (eps device and eps_host host)
 *   W_host          host array of n_k device pointers: W(t) [n_mesh][N][N]
 *                   c128 for transfer t, e.g. gw_screen of the polarization
 *                   whose kq_host is (k + t) mod n_k
 *   v               device [N] FP64 Coulomb diagonal
 *   sigma           device [n_states][n_out] c128, overwritten
 * Workspace from gw_sigma_c_workspace_size; errors as for gw_polarization. */
typedef struct {
  int precision, n_k, N, R, n_bands;
  int n_mesh;
  const double* mesh_host;
  int n_out;
  const double* omega_out_host;
  int n_states;
  const int* state_set_host;
  const int* state_band_host;
  double mu;
  const void* U;
  const void* psi;
  const double* eps;
  const double* eps_host;
  const void* const* W_host;
  const double* v;
  void* sigma;
} gw_sigma_desc;

int gw_sigma_c_workspace_size(const gw_sigma_desc* d_host, size_t* bytes);
int gw_sigma_c(void* stream, const gw_sigma_desc* d_host, void* ws, size_t ws_bytes);

/* --------------------------------------------------------------------- tuning
 * Process-wide kernel-variant switches for the split-BF16 path (all results
 * stay within the same tolerances; the work done is identical).  Keys:
 *   "bf16_pipeline"       1: pair products (Eq. proj_MB) formed and split in
 *                         registers while the projection kernel stages its
 *                         tiles, weights applied while the accumulation
 *                         kernel stages its tiles;
 *                         2 (default): streaming kernels write the split,
 *                         sign-patterned operand words (U once per call, the
 *                         products and the weighted projections per chunk)
 *                         in the tiled layout of one shared MFMA GEMM core.
 *   "projection_variant"  pipeline 1 only, N >= 256: 1: 128 x 128 output
 *                         tiles; 2 (default): 256 x 128 output tiles with the
 *                         staging of the next K stage interleaved with the
 *                         MFMAs.
 *   "gemm_staging"        pipeline 2 with complex_product 4: 1: 4 waves,
 *                         operand stages pass through registers into LDS; 2:
 *                         4 waves, direct global-to-LDS copies; 3 (default):
 *                         8 waves (two per SIMD), register staging; 4: 8 waves
 *                         in ping-pong (the two waves of a SIMD alternate
 *                         between MFMAs and memory work; same results bit for
 *                         bit).
 *   "fp16_core"           GW_SPLIT_FP16: 1 (default): operands staged inside
 *                         the GEMM kernels, lo words pre-scaled by 2^11 in a
 *                         separate accumulator (FP32-level accuracy); 2: the
 *                         three-multiplication core below on plane words with
 *                         power-of-two row / pair scales (hi in [2^13, 2^14))
 *                         and one accumulator set: twice as fast, the
 *                         accuracy of split BF16 (the FP32 accumulation of the
 *                         three products per accumulator dominates).
 *   "complex_product"     pipeline 2: 3 (default): every complex product of
 *                         the projection and the accumulation as three real
 *                         products (Gauss: T1 = ac, T2 = bd, T3 = (a+b)(c+d);
 *                         Re = T1 - T2, Im = T3 - T1 - T2) on real operand
 *                         planes, 8 waves, operands copied straight into LDS,
 *                         a quarter fewer MFMAs; 4: four real products per
 *                         complex product (the gemm_staging variants above).
 *   "gemm3m_pipeline"     staging of the three-multiplication core: 6
 *                         (default): six 24 KB LDS slots, one plane (hi and lo
 *                         words of A and of both B halves) each, copied
 *                         gemm3m_lead plane steps before use, one barrier per
 *                         plane step; 2: two 72 KB stage buffers, the next
 *                         stage copied while the current one is multiplied,
 *                         one barrier per stage.  Same results bit for bit.
 *   "gemm3m_lead"         six-slot staging: 3, 4 (default) or 5 plane steps
 *                         between a slot's copy and its use.  Same results
 *                         bit for bit.
 *   "real_core"           real inputs (gw_pol_desc.real_inputs): 1: the
 *                         8-wave core with operands staged through registers;
 *                         2 (default): the six-slot core, a real stage of 32 k
 *                         taken as two planes of 16 k into one accumulator
 *                         set.  Same results bit for bit.
 * Values out of range and unknown keys give GW_ERR_INVALID_ARG.  Not
 * thread-safe: set before launching work.  gw_get_tuning reads a key's
 * current value. */
int gw_set_tuning(const char* key_host, int value);
int gw_get_tuning(const char* key_host, int* value_host);

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
