// Learned high-band correction of P (features, training targets, application,
// judge).  The unoccupied bands above a cutoff are left out of the explicit sum
// of Eq. polar_MB; a perceptron predicts, per basis function I and frequency,
// the log-ratio y of the missing diagonal d_I to the retained diagonal
// |P_ret,II|, and the correction is the congruence
//     P = P_ret + D P_ret D,   D = diag(exp(y/2)),
// which adds exactly -d_I on the diagonal and keeps P Hermitian and negative
// semidefinite.  (The paper corrects the same band truncation with the
// extrapolar approximation; this model learns the correction from full-band
// runs instead.)
#include <algorithm>
#include <cmath>

#include "gw_internal.hpp"

namespace gw {
namespace {

constexpr int kMaxK = 64;
constexpr int kMaxRows = 64;
constexpr int NF = 12;  // features used (rest of the row is zero)
inline int cdiv_int(long a, long b) { return (int)((a + b - 1) / b); }

struct KMap {
  int n_k;
  int kq[kMaxK];
};
// Optional explicit list of (k, n) occupied rows; n = 0 means all k x occupied.
struct RowList {
  int n;
  int k[kMaxRows];
  int o[kMaxRows];
};

// Partial sums over unoccupied bands of |w| = 4|D|/(D^2 + w^2) for one
// occupied row per block, split at the cutoff: out[blk][j][0] (< cut), [1] (>= cut).
__global__ __launch_bounds__(256) void wsum_kernel(const double* __restrict__ eps, int n_occ, int n_unocc, int cut,
                                                   KMap km, RowList rl, OmegaList om, double* __restrict__ part) {
  __shared__ double red[256];
  int k, n;
  if (rl.n > 0) {
    k = rl.k[blockIdx.x];
    n = rl.o[blockIdx.x];
  } else {
    k = blockIdx.x / n_occ;
    n = blockIdx.x % n_occ;
  }
  const int nb = n_occ + n_unocc;
  const double eo = eps[(size_t)k * nb + n];
  const double* eu = eps + (size_t)km.kq[k] * nb + n_occ;
  for (int j = 0; j < om.n; ++j) {
    double w2 = om.w[j] * om.w[j];
    double lo = 0.0, hi = 0.0;
    for (int u = threadIdx.x; u < n_unocc; u += 256) {
      double d = fabs(eo - eu[u]);
      double x = 4.0 * d / (d * d + w2);
      if (u < cut) lo += x;
      else hi += x;
    }
    for (int half = 0; half < 2; ++half) {
      red[threadIdx.x] = half ? hi : lo;
      __syncthreads();
      for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[((size_t)blockIdx.x * om.n + j) * 2 + half] = red[0];
      __syncthreads();
    }
  }
}

// sums[j][h] = sum over blocks of part (fixed order).
__global__ void wsum_final_kernel(int nblk, int n_om, const double* __restrict__ part, double* __restrict__ sums) {
  int e = threadIdx.x;
  if (e >= 2 * n_om) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * 2 * n_om + e];
  sums[e] = s;
}

// Band-edge energies averaged over k-sets: [0] lowest occupied, [1] highest
// occupied, [2] lowest unoccupied, [3] highest retained unoccupied, [4] highest unoccupied.
__global__ void edges_kernel(const double* __restrict__ eps, int n_k, int n_occ, int n_unocc, int cut,
                             double* __restrict__ edges) {
  if (threadIdx.x != 0) return;
  const int nb = n_occ + n_unocc;
  double s[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < n_k; ++k) {
    const double* e = eps + (size_t)k * nb;
    s[0] += e[0];
    s[1] += e[n_occ - 1];
    s[2] += e[n_occ];
    s[3] += e[n_occ + cut - 1];
    s[4] += e[nb - 1];
  }
  for (int i = 0; i < 5; ++i) edges[i] = s[i] / n_k;
}

// mean over I of |Re P_j[I][I]| per frequency (fixed-order block reduction).
__global__ __launch_bounds__(256) void diagmean_kernel(int N, const double2* __restrict__ P, double* __restrict__ mean) {
  __shared__ double red[256];
  const double2* Pj = P + (size_t)blockIdx.x * N * N;
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) s += fabs(Pj[(size_t)i * N + i].x);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[blockIdx.x] = red[0] / N;
}

__device__ inline double safe_log(double x) { return log(fmax(x, 1e-300)); }

// Feature rows r = j*N + I (frequency-major).
__global__ void features_kernel(int N, OmegaList om, int cut, int n_unocc, const double2* __restrict__ P,
                                const double* __restrict__ sums, const double* __restrict__ edges,
                                const double* __restrict__ mean, int n_in, float* __restrict__ X) {
  size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (r >= (size_t)N * om.n) return;
  const int j = (int)(r / N), I = (int)(r % N);
  const double w = om.w[j];
  const double p = fabs(P[((size_t)j * N + I) * N + I].x);
  const double p0 = fabs(P[(size_t)I * N + I].x);
  const double lo = sums[2 * j], hi = sums[2 * j + 1];
  const double lo0 = sums[0], hi0 = sums[1];
  float f[NF];
  f[0] = (float)(w / (1.0 + w));
  f[1] = (float)(safe_log(hi) - safe_log(lo));
  f[2] = (float)(safe_log(p) - safe_log(p0));
  f[3] = (float)(safe_log(p) - safe_log(mean[j]));
  f[4] = (float)I / (float)N;
  f[5] = (float)(edges[3] - edges[2]);
  f[6] = (float)(edges[4] - edges[3]);
  f[7] = (float)(edges[1] - edges[0]);
  f[8] = (float)(edges[2] - edges[1]);
  f[9] = (float)cut / (float)n_unocc;
  f[10] = f[1] - (float)(safe_log(hi0) - safe_log(lo0));
  f[11] = (float)(safe_log(lo) - safe_log(lo0));
  float* xr = X + r * n_in;
  for (int c = 0; c < n_in; ++c) xr[c] = c < NF ? f[c] : 0.f;
}

// t = log(d / |P_ret,II|), d = Re P_ret,II - Re P_full,II (> 0 when bands were left out).
__global__ void targets_kernel(int N, int n_om, const double2* __restrict__ Pr, const double2* __restrict__ Pf,
                               float* __restrict__ T, float* __restrict__ mask) {
  size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (r >= (size_t)N * n_om) return;
  const int j = (int)(r / N), I = (int)(r % N);
  const size_t o = ((size_t)j * N + I) * N + I;
  double pr = fabs(Pr[o].x);
  double d = Pr[o].x - Pf[o].x;
  bool ok = pr > 0.0 && d > 0.0 && isfinite(d);
  T[r] = ok ? (float)log(d / pr) : 0.f;
  mask[r] = ok ? 1.f : 0.f;
}

__device__ inline double yclamp(float y) { return fmin(fmax((double)y, -30.0), 30.0); }

// P_j[I][J] *= 1 + exp((y_I + y_J)/2)  (i.e. P + D P D).
__global__ void apply_kernel(int N, int n_om, const float* __restrict__ Y, int ldy, double2* __restrict__ P) {
  const size_t NN = (size_t)N * N;
  const size_t total = NN * n_om;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / NN);
    const size_t q = e % NN;
    const int I = (int)(q / N), J = (int)(q % N);
    double yi = yclamp(Y[((size_t)j * N + I) * ldy]);
    double yj = yclamp(Y[((size_t)j * N + J) * ldy]);
    double f = 1.0 + exp(0.5 * (yi + yj));
    double2 p = P[e];
    P[e] = make_double2(p.x * f, p.y * f);
  }
}

// Judge: relative difference between the predicted missing trace and the
// trace of an explicitly summed sample of left-out transitions scaled by the
// sample's share of the left-out weight: err_j = |TRs/f - TRp| / TRp.
__global__ __launch_bounds__(256) void judge_kernel(int N, const float* __restrict__ Y, int ldy,
                                                    const double2* __restrict__ Pr, const double2* __restrict__ Ps,
                                                    const double* __restrict__ all_sums,
                                                    const double* __restrict__ sample_sums,
                                                    double* __restrict__ err) {
  __shared__ double ra[256], rb[256];
  const int j = blockIdx.x;
  const double2* Prj = Pr + (size_t)j * N * N;
  const double2* Psj = Ps + (size_t)j * N * N;
  double tp = 0.0, ts = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) {
    tp += fabs(Prj[(size_t)i * N + i].x) * exp(yclamp(Y[((size_t)j * N + i) * ldy]));
    ts += fabs(Psj[(size_t)i * N + i].x);
  }
  ra[threadIdx.x] = tp;
  rb[threadIdx.x] = ts;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ra[threadIdx.x] += ra[threadIdx.x + w];
      rb[threadIdx.x] += rb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double f = sample_sums[2 * j + 1] / all_sums[2 * j + 1];
    double est = rb[0] / f;
    err[j] = fabs(est - ra[0]) / fmax(ra[0], 1e-300);
  }
}

// Left-out trace of one judge sample row (k, n) from its projections M
// [N][ldm] (columns t < nu: the unoccupied bands cut.. of set kq):
//   TR_j = sum_I |Re P_II| = sum_t |w_t(j)| sum_I |M_It|^2,
// since every w_t(j) = 4 D_t / (D_t^2 + w_j^2) < 0.  Block (x, y) covers
// columns 256 x .. and rows 256 y ..; its partial sums per frequency go to
// part[(y * gridDim.x + x) * n_omega + j] (fixed-order tree in LDS).
template <class CT>
__global__ __launch_bounds__(256) void sample_trace_kernel(const CT* __restrict__ M, int N, int nu, long ldm,
                                                           const double* __restrict__ eo,
                                                           const double* __restrict__ eu, OmegaList om,
                                                           double* __restrict__ part) {
  __shared__ double red[256];
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int i0 = blockIdx.y * 256, i1 = min(N, i0 + 256);
  double c = 0.0;
  if (t < nu)
    for (int I = i0; I < i1; ++I) {
      const CT m = M[(size_t)I * ldm + t];
      c += (double)m.x * (double)m.x + (double)m.y * (double)m.y;
    }
  const double d = t < nu ? eo[0] - eu[t] : -1.0;
  double* out = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * om.n;
  for (int j = 0; j < om.n; ++j) {
    red[threadIdx.x] = t < nu ? c * fabs(4.0 * d / (d * d + om.w[j] * om.w[j])) : 0.0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
    __syncthreads();
  }
}

// trs[j] = sum over p < n_part of part[p * n_om + j], in order.
__global__ void trace_final_kernel(int n_part, int n_om, const double* __restrict__ part, double* __restrict__ trs) {
  const int j = threadIdx.x;
  if (j >= n_om) return;
  double s = 0.0;
  for (int p = 0; p < n_part; ++p) s += part[(size_t)p * n_om + j];
  trs[j] = s;
}

// Judge from the sample's left-out trace trs (see judge_kernel).
__global__ __launch_bounds__(256) void judge_tr_kernel(int N, const float* __restrict__ Y, int ldy,
                                                       const double2* __restrict__ Pr,
                                                       const double* __restrict__ trs,
                                                       const double* __restrict__ all_sums,
                                                       const double* __restrict__ sample_sums,
                                                       double* __restrict__ err) {
  __shared__ double ra[256];
  const int j = blockIdx.x;
  const double2* Prj = Pr + (size_t)j * N * N;
  double tp = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) tp += fabs(Prj[(size_t)i * N + i].x) * exp(yclamp(Y[((size_t)j * N + i) * ldy]));
  ra[threadIdx.x] = tp;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) ra[threadIdx.x] += ra[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double f = sample_sums[2 * j + 1] / all_sums[2 * j + 1];
    err[j] = fabs(trs[j] / f - ra[0]) / fmax(ra[0], 1e-300);
  }
}

int fill_kmap(int n_k, const int* kq_host, KMap& km) {
  if (n_k > kMaxK) return fail(GW_ERR_UNSUPPORTED, "surrogate: at most 64 k-sets");
  km.n_k = n_k;
  for (int k = 0; k < kMaxK; ++k) km.kq[k] = k < n_k ? (kq_host ? kq_host[k] : (k + 1) % n_k) : 0;
  for (int k = 0; k < n_k; ++k)
    if (km.kq[k] < 0 || km.kq[k] >= n_k) return fail(GW_ERR_INVALID_ARG, "surrogate: kq entry out of range");
  return GW_OK;
}

int fill_omega(int n, const double* w, OmegaList& om) {
  if (n < 1 || n > kMaxOmega || !w) return fail(GW_ERR_INVALID_ARG, "surrogate: 1..64 frequencies required");
  om.n = n;
  for (int j = 0; j < kMaxOmega; ++j) {
    om.w[j] = j < n ? w[j] : 0.0;
    if (j < n && !(std::isfinite(w[j]) && w[j] >= 0.0))
      return fail(GW_ERR_INVALID_ARG, "surrogate: frequencies must be finite and >= 0");
  }
  return GW_OK;
}

int check_desc(const gw_surr_desc* d) {
  if (!d) return fail(GW_ERR_INVALID_ARG, "surrogate: desc is NULL");
  if (d->N < 1 || d->n_k < 1 || d->n_occ < 1 || d->n_unocc < 1 || d->cut < 1 || d->cut > d->n_unocc)
    return fail(GW_ERR_INVALID_ARG, "surrogate: need N, n_k, n_occ, n_unocc >= 1 and 1 <= cut <= n_unocc");
  if (!d->eps || !d->P_ret) return fail(GW_ERR_INVALID_ARG, "surrogate: eps and P_ret are required");
  if (d->n_in < NF || d->n_in % 32 != 0) return fail(GW_ERR_INVALID_ARG, "surrogate: n_in must be >= 12 and a multiple of 32");
  return GW_OK;
}

size_t wsum_part_bytes(int rows, int n_om) { return align_up((size_t)rows * n_om * 2 * sizeof(double)); }

int run_wsum(hipStream_t s, const gw_surr_desc& d, const KMap& km, const RowList& rl, const OmegaList& om,
             double* part, double* sums) {
  int nblk = rl.n > 0 ? rl.n : d.n_k * d.n_occ;
  hipLaunchKernelGGL(wsum_kernel, dim3(nblk), dim3(256), 0, s, d.eps, d.n_occ, d.n_unocc, d.cut, km, rl, om, part);
  GW_LAUNCHED("wsum_kernel");
  hipLaunchKernelGGL(wsum_final_kernel, dim3(1), dim3(128), 0, s, nblk, om.n, part, sums);
  GW_LAUNCHED("wsum_final_kernel");
  return GW_OK;
}

}  // namespace

int sample_trace_parts(int N, int nu) { return cdiv_int(N, 256) * cdiv_int(nu, 256); }

int launch_sample_trace(hipStream_t s, bool c128, const void* M, int N, int nu, long ldm, const double* eo,
                        const double* eu, const OmegaList& om, double* part) {
  dim3 grid(cdiv_int(nu, 256), cdiv_int(N, 256));
  if (c128)
    hipLaunchKernelGGL(sample_trace_kernel<double2>, grid, dim3(256), 0, s, static_cast<const double2*>(M), N, nu,
                       ldm, eo, eu, om, part);
  else
    hipLaunchKernelGGL(sample_trace_kernel<float2>, grid, dim3(256), 0, s, static_cast<const float2*>(M), N, nu,
                       ldm, eo, eu, om, part);
  GW_LAUNCHED("sample_trace_kernel");
  return GW_OK;
}

int surrogate_judge_traces(hipStream_t s, const gw_surr_desc& d, const float* Y, int ldy, const double* part,
                           int n_part, int n_rows, const int* rk, const int* ro, double* err, void* ws) {
  OmegaList om;
  KMap km;
  int st;
  if ((st = fill_omega(d.n_omega, d.omega_host, om)) != GW_OK) return st;
  if ((st = fill_kmap(d.n_k, d.kq_host, km)) != GW_OK) return st;
  if (n_rows < 1 || n_rows > kMaxRows) return fail(GW_ERR_INVALID_ARG, "judge: 1..64 sample rows");
  RowList rl;
  rl.n = n_rows;
  for (int i = 0; i < kMaxRows; ++i) {
    rl.k[i] = i < n_rows ? rk[i] : 0;
    rl.o[i] = i < n_rows ? ro[i] : 0;
  }
  Carver cv(ws);
  double* wpart = cv.take<double>((size_t)std::max(d.n_k * d.n_occ, kMaxRows) * d.n_omega * 2);
  double* sums = cv.take<double>(2 * kMaxOmega);
  double* ssum = cv.take<double>(2 * kMaxOmega);
  double* trs = cv.take<double>(2 * kMaxOmega);
  RowList all;
  all.n = 0;
  if ((st = run_wsum(s, d, km, all, om, wpart, sums)) != GW_OK) return st;
  if ((st = run_wsum(s, d, km, rl, om, wpart, ssum)) != GW_OK) return st;
  hipLaunchKernelGGL(trace_final_kernel, dim3(1), dim3(64), 0, s, n_part, d.n_omega, part, trs);
  GW_LAUNCHED("trace_final_kernel");
  hipLaunchKernelGGL(judge_tr_kernel, dim3(d.n_omega), dim3(256), 0, s, d.N, Y, ldy,
                     reinterpret_cast<const double2*>(d.P_ret), trs, sums, ssum, err);
  GW_LAUNCHED("judge_tr_kernel");
  return GW_OK;
}

}  // namespace gw

using namespace gw;

extern "C" {

int gw_surrogate_workspace_size(const gw_surr_desc* d, size_t* bytes) {
  int st = check_desc(d);
  if (st != GW_OK) return st;
  if (!bytes) return fail(GW_ERR_INVALID_ARG, "gw_surrogate_workspace_size: bytes_host is NULL");
  *bytes = wsum_part_bytes(std::max(d->n_k * d->n_occ, kMaxRows), d->n_omega) + 3 * align_up(2 * kMaxOmega * sizeof(double)) +
           align_up(8 * sizeof(double)) + align_up(kMaxOmega * sizeof(double));
  return GW_OK;
}

int gw_surrogate_features(void* stream, const gw_surr_desc* d, float* X, void* ws, size_t ws_bytes) {
  int st = check_desc(d);
  if (st != GW_OK) return st;
  if (!X) return fail(GW_ERR_INVALID_ARG, "gw_surrogate_features: X is NULL");
  size_t need = 0;
  gw_surrogate_workspace_size(d, &need);
  if (!ws || ws_bytes < need) return fail(GW_ERR_WORKSPACE, "gw_surrogate_features: workspace too small");
  OmegaList om;
  KMap km;
  if ((st = fill_omega(d->n_omega, d->omega_host, om)) != GW_OK) return st;
  if ((st = fill_kmap(d->n_k, d->kq_host, km)) != GW_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(ws);
  double* part = cv.take<double>((size_t)std::max(d->n_k * d->n_occ, kMaxRows) * d->n_omega * 2);
  double* sums = cv.take<double>(2 * kMaxOmega);
  cv.take<double>(2 * kMaxOmega);
  cv.take<double>(2 * kMaxOmega);
  double* edges = cv.take<double>(8);
  double* mean = cv.take<double>(kMaxOmega);
  RowList all;
  all.n = 0;
  if ((st = run_wsum(s, *d, km, all, om, part, sums)) != GW_OK) return st;
  hipLaunchKernelGGL(edges_kernel, dim3(1), dim3(64), 0, s, d->eps, d->n_k, d->n_occ, d->n_unocc, d->cut, edges);
  GW_LAUNCHED("edges_kernel");
  const double2* P = reinterpret_cast<const double2*>(d->P_ret);
  hipLaunchKernelGGL(diagmean_kernel, dim3(d->n_omega), dim3(256), 0, s, d->N, P, mean);
  GW_LAUNCHED("diagmean_kernel");
  size_t rows = (size_t)d->N * d->n_omega;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, d->N, om, d->cut,
                     d->n_unocc, P, sums, edges, mean, d->n_in, X);
  GW_LAUNCHED("features_kernel");
  return GW_OK;
}

int gw_surrogate_targets(void* stream, int N, int n_omega, const double* P_ret, const double* P_full, float* T,
                         float* mask) {
  if (N < 1 || n_omega < 1 || !P_ret || !P_full || !T || !mask)
    return fail(GW_ERR_INVALID_ARG, "gw_surrogate_targets: bad arguments");
  size_t rows = (size_t)N * n_omega;
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), N, n_omega, reinterpret_cast<const double2*>(P_ret),
                     reinterpret_cast<const double2*>(P_full), T, mask);
  GW_LAUNCHED("targets_kernel");
  return GW_OK;
}

int gw_surrogate_apply(void* stream, int N, int n_omega, const float* Y, int ldy, double* P) {
  if (N < 1 || n_omega < 1 || !Y || !P || ldy < 1) return fail(GW_ERR_INVALID_ARG, "gw_surrogate_apply: bad arguments");
  size_t total = (size_t)N * N * n_omega;
  unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 65536);
  ProfScope prof(static_cast<hipStream_t>(stream), "apply_kernel");
  hipLaunchKernelGGL(apply_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), N, n_omega, Y, ldy,
                     reinterpret_cast<double2*>(P));
  GW_LAUNCHED("apply_kernel");
  return GW_OK;
}

int gw_surrogate_judge(void* stream, const gw_surr_desc* d, const float* Y, int ldy, const double* P_sample,
                       int n_sample, const int* sample_k_host, const int* sample_occ_host, double* err, void* ws,
                       size_t ws_bytes) {
  int st = check_desc(d);
  if (st != GW_OK) return st;
  if (!Y || ldy < 1 || !P_sample || !err || n_sample < 1 || n_sample > kMaxRows || !sample_k_host || !sample_occ_host)
    return fail(GW_ERR_INVALID_ARG, "gw_surrogate_judge: bad arguments (1..64 sample rows)");
  size_t need = 0;
  gw_surrogate_workspace_size(d, &need);
  if (!ws || ws_bytes < need) return fail(GW_ERR_WORKSPACE, "gw_surrogate_judge: workspace too small");
  OmegaList om;
  KMap km;
  if ((st = fill_omega(d->n_omega, d->omega_host, om)) != GW_OK) return st;
  if ((st = fill_kmap(d->n_k, d->kq_host, km)) != GW_OK) return st;
  RowList rl;
  rl.n = n_sample;
  for (int i = 0; i < kMaxRows; ++i) {
    rl.k[i] = i < n_sample ? sample_k_host[i] : 0;
    rl.o[i] = i < n_sample ? sample_occ_host[i] : 0;
    if (i < n_sample && (rl.k[i] < 0 || rl.k[i] >= d->n_k || rl.o[i] < 0 || rl.o[i] >= d->n_occ))
      return fail(GW_ERR_INVALID_ARG, "gw_surrogate_judge: sample row out of range");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(ws);
  double* part = cv.take<double>((size_t)std::max(d->n_k * d->n_occ, kMaxRows) * d->n_omega * 2);
  double* sums = cv.take<double>(2 * kMaxOmega);
  double* ssum = cv.take<double>(2 * kMaxOmega);
  RowList all;
  all.n = 0;
  if ((st = run_wsum(s, *d, km, all, om, part, sums)) != GW_OK) return st;
  if ((st = run_wsum(s, *d, km, rl, om, part, ssum)) != GW_OK) return st;
  hipLaunchKernelGGL(judge_kernel, dim3(d->n_omega), dim3(256), 0, s, d->N, Y, ldy,
                     reinterpret_cast<const double2*>(d->P_ret), reinterpret_cast<const double2*>(P_sample), sums,
                     ssum, err);
  GW_LAUNCHED("judge_kernel");
  return GW_OK;
}

}  // extern "C"
