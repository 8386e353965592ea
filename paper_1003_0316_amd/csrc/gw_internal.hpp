// Internal declarations shared by the libgw translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/gw.h"

namespace gw {

// ---- error reporting ---------------------------------------------------------
int fail(int status, const std::string& msg);          // records msg, returns status
int hip_fail(hipError_t e, const char* what);          // GW_ERR_HIP with the HIP message
#define GW_HIP(call)                                          \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::gw::hip_fail(e_, #call);   \
  } while (0)
#define GW_LAUNCHED(what)                                     \
  do {                                                        \
    hipError_t e_ = hipGetLastError();                        \
    if (e_ != hipSuccess) return ::gw::hip_fail(e_, what);    \
  } while (0)

constexpr int kMaxOmega = 64;   // imaginary frequencies per call
constexpr int kMaxSlots = 256;  // accumulation slots: frequencies, or the energy nodes of the spectral route
// The slots a polarization pass accumulates into.  hat == 0: slot j is the
// imaginary frequency w[j]; hat == 1: slot j is the transition-energy node
// w[j] of the spectral route (increasing).
struct OmegaList {
  int n;
  int hat = 0;
  double w[kMaxSlots];
};

// Weight of a transition with D = e_occ - e_unocc < 0 in slot j: the
// spin-summed imaginary-axis bracket of Eq. polar_MB, 4 D / (D^2 + w_j^2), or,
// on the spectral route, minus the share of the transition's spectral weight
// that goes to node j when it is split linearly between the two nodes around
// x = -D.
__device__ inline double pair_weight(double d, const OmegaList& om, int j) {
  if (!om.hat) return 4.0 * d / (d * d + om.w[j] * om.w[j]);
  const double x = -d, xj = om.w[j];
  if (j > 0 && x >= om.w[j - 1] && x <= xj) return -(x - om.w[j - 1]) / (xj - om.w[j - 1]);
  if (j + 1 < om.n && x > xj && x <= om.w[j + 1]) return -(om.w[j + 1] - x) / (om.w[j + 1] - xj);
  if (j == 0 && x == xj) return -1.0;
  return 0.0;
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Workspace carving helper: hands out 256-byte aligned slices of one buffer.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

// ---- optional launch timing (gw_profile_*) ----------------------------------------
class ProfScope {
 public:
  ProfScope(hipStream_t s, const char* name);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  hipStream_t s_;
  const char* name_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  bool active_ = false;
};

// ---- transition-pair chunk ---------------------------------------------------
// A chunk is a run of T consecutive transition pairs of set k (occupied) and
// set kq (unoccupied).  The pairs of a call form the grid (n, n') with n from
// n0 and n' from u0 (u0 counts from the first unoccupied band) and nu
// unoccupied bands per row; chunk pair t is grid index g = tb + t, i.e.
// n = n0 + g / nu, n' = u0 + g % nu.
struct Chunk {
  int k, kq;
  int n0, u0, nu;
  long tb;
  int T;
  int pairs() const { return T; }
};

// ---- spectral route (k_fp64.hip) -------------------------------------------------
// P[j] (+)= sum_b 4 x_b / (x_b^2 + omega_j^2) S[b] over all N x N elements; S
// holds the node accumulations (-S_b), [n_nodes][N][N].
int launch_spectral_combine(hipStream_t s, int N, const OmegaList& nodes, int n_omega, const double* omega_host,
                            const double2* S, double2* P, int accumulate);

// ---- FP64 path (k_fp64.hip) ----------------------------------------------------
int launch_fill_zero(hipStream_t s, double* p, size_t n_doubles);
int launch_weights_f64(hipStream_t s, const double* eps, int n_bands, int n_occ, const Chunk& c,
                       const OmegaList& om, double* w /*[n_omega][pairs]*/);
int launch_project_f64(hipStream_t s, int N, int R, const double2* U, const double2* psi_occ,
                       const double2* psi_unocc, int nu, long tb, int T, double2* M, long ldm);
int launch_herk_f64(hipStream_t s, int N, int T, const double2* M, long ldm, const double* w,
                    int n_omega, double2* P);
int launch_hermitian_mirror(hipStream_t s, int N, int n_omega, double2* P);

// ---- finite checks (k_fp64.hip) ---------------------------------------------
constexpr size_t kFlagBytes = 256;  // one device flag at the end of a workspace
int launch_flag_clear(hipStream_t s, unsigned* flag);
// flag |= 1 if any of n_values floats (or doubles when f64) is Inf or NaN.
int launch_nonfinite(hipStream_t s, const void* p, size_t n_values, bool f64, unsigned* flag);
// Copies the flag to the host and synchronises the stream.
int read_flag(hipStream_t s, const unsigned* flag, unsigned* host);

// ---- learned correction (k_surrogate.hip) ------------------------------------
// Partial sums per sample row of launch_sample_trace, per frequency.
int sample_trace_parts(int N, int nu);
// Left-out trace partials of one judge sample row from its projections M
// [N][ldm] (c128 or c64), columns t < nu with energies eu[t], occupied energy
// *eo: part[p][j] for p < sample_trace_parts(N, nu).
int launch_sample_trace(hipStream_t s, bool c128, const void* M, int N, int nu, long ldm, const double* eo,
                        const double* eu, const OmegaList& om, double* part);
// err[j] from the predicted left-out trace (P_ret, Y) and the sample's traces
// (n_part partials per frequency, summed in order), scaled by the sample rows'
// share of the left-out weight sum.  ws: gw_surrogate_workspace_size bytes.
int surrogate_judge_traces(hipStream_t s, const gw_surr_desc& d, const float* Y, int ldy, const double* part,
                           int n_part, int n_rows, const int* rk, const int* ro, double* err, void* ws);

// ---- screening (k_screen.hip) ---------------------------------------------------
size_t screen_workspace_bytes(int N, int n_omega);
int screen_run(hipStream_t s, int N, int n_omega, const double2* P, const double* v, double2* W,
               int* info, void* ws);

}  // namespace gw
