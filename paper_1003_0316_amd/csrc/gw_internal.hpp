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

constexpr int kMaxOmega = 64;
struct OmegaList {
  int n;
  double w[kMaxOmega];
};

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

// ---- FP64 path (k_fp64.hip) ----------------------------------------------------
int launch_fill_zero(hipStream_t s, double* p, size_t n_doubles);
int launch_weights_f64(hipStream_t s, const double* eps, int n_bands, int n_occ, const Chunk& c,
                       const OmegaList& om, double* w /*[n_omega][pairs]*/);
int launch_project_f64(hipStream_t s, int N, int R, const double2* U, const double2* psi_occ,
                       const double2* psi_unocc, int nu, long tb, int T, double2* M, long ldm);
int launch_herk_f64(hipStream_t s, int N, int T, const double2* M, long ldm, const double* w,
                    int n_omega, double2* P);
int launch_hermitian_mirror(hipStream_t s, int N, int n_omega, double2* P);

// ---- screening (k_screen.hip) ---------------------------------------------------
size_t screen_workspace_bytes(int N, int n_omega);
int screen_run(hipStream_t s, int N, int n_omega, const double2* P, const double* v, double2* W,
               int* info, void* ws);

}  // namespace gw
