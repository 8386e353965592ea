// libgw C ABI: argument validation, workspace planning, chunk loop.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "gw_internal.hpp"
#include "gw_mfma.hpp"

namespace gw {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return GW_ERR_HIP;
}

namespace {

bool valid_precision(int p) { return p >= GW_FP64 && p <= GW_SPLIT_FP16; }
size_t cplx_bytes(int p) { return p == GW_FP64 ? 16 : 8; }

// Chunk size for one polarization call.
struct Plan {
  int tc = 0;     // max pairs per chunk
  size_t ws = 0;  // workspace bytes
};

int default_chunk_pairs(const gw_pol_desc& d) {
  if (d.chunk_pairs > 0) return d.chunk_pairs;
  if (d.precision == GW_FP64) {
    size_t target = (size_t)128 << 20;  // M chunk bytes
    size_t p = target / ((size_t)d.N * 16);
    return (int)std::max<size_t>(64, std::min<size_t>(p, 65536));
  }
  return mfma_default_chunk_pairs(d.N, d.R, d.n_omega, d.precision);
}

// The polarization pass of the spectral route: the node energies are its
// accumulation slots, the node matrices (in the workspace) its output.
gw_pol_desc spectral_inner(const gw_pol_desc& d, double2* S) {
  gw_pol_desc in = d;
  in.n_omega = d.n_nodes;
  in.omega_host = d.nodes_host;
  in.P = reinterpret_cast<double*>(S);
  in.accumulate = 0;
  in.n_nodes = 0;
  in.nodes_host = nullptr;
  return in;
}

size_t node_bytes(const gw_pol_desc& d) { return align_up((size_t)d.n_nodes * d.N * d.N * 16); }

Plan make_plan_direct(const gw_pol_desc& d);

Plan make_plan(const gw_pol_desc& d) {
  if (d.n_nodes > 0) {
    Plan pl = make_plan_direct(spectral_inner(d, nullptr));
    pl.ws += node_bytes(d);
    return pl;
  }
  return make_plan_direct(d);
}

Plan make_plan_direct(const gw_pol_desc& d) {
  Plan pl;
  const long total = (long)(d.occ_end - d.occ_begin) * (d.unocc_end - d.unocc_begin);
  pl.tc = (int)std::max(1L, std::min<long>(default_chunk_pairs(d), total));
  if (d.precision == GW_FP64) {
    pl.ws = align_up((size_t)d.N * pl.tc * 16) + align_up((size_t)d.n_omega * pl.tc * sizeof(double));
  } else {
    pl.ws = d.real_inputs ? tiled_pol_workspace_real(d.N, d.R, pl.tc, d.n_omega)
                          : mfma_pol_workspace(d.precision, d.N, d.R, pl.tc, d.n_omega);
  }
  return pl;
}

int validate_desc(const gw_pol_desc* dp) {
  if (!dp) return fail(GW_ERR_INVALID_ARG, "gw_polarization: desc is NULL");
  const gw_pol_desc& d = *dp;
  if (!valid_precision(d.precision)) return fail(GW_ERR_INVALID_ARG, "gw_polarization: unknown precision");
  if (d.real_inputs != 0 && d.real_inputs != 1)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization: real_inputs must be 0 or 1");
  if (d.real_inputs && d.precision != GW_SPLIT_BF16)
    return fail(GW_ERR_UNSUPPORTED, "gw_polarization: real inputs are supported with GW_SPLIT_BF16 only");
  if (d.n_k < 1 || d.N < 1 || d.R < 1 || d.n_occ < 1 || d.n_unocc < 1 || d.n_omega < 1)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization: n_k, N, R, n_occ, n_unocc, n_omega must be >= 1");
  if (d.n_omega > kMaxOmega)
    return fail(GW_ERR_UNSUPPORTED, "gw_polarization: at most 64 frequencies per call");
  if (d.occ_begin < 0 || d.occ_end > d.n_occ || d.occ_begin >= d.occ_end)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization: need 0 <= occ_begin < occ_end <= n_occ");
  if (d.unocc_begin < 0 || d.unocc_end > d.n_unocc || d.unocc_begin >= d.unocc_end)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization: need 0 <= unocc_begin < unocc_end <= n_unocc");
  if (!d.omega_host || !d.U || !d.psi || !d.eps || !d.eps_host || !d.P)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization: null pointer among omega_host, U, psi, eps, eps_host, P");
  if (d.chunk_pairs < 0) return fail(GW_ERR_INVALID_ARG, "gw_polarization: chunk_pairs < 0");
  if ((long long)d.N * d.N > (1LL << 31) || (long long)d.N * d.R > (1LL << 40))
    return fail(GW_ERR_UNSUPPORTED, "gw_polarization: problem too large");
  for (int j = 0; j < d.n_omega; ++j)
    if (!std::isfinite(d.omega_host[j]) || d.omega_host[j] < 0.0)
      return fail(GW_ERR_INVALID_ARG, "gw_polarization: frequencies must be finite and >= 0");
  if (d.kq_host)
    for (int k = 0; k < d.n_k; ++k)
      if (d.kq_host[k] < 0 || d.kq_host[k] >= d.n_k)
        return fail(GW_ERR_INVALID_ARG, "gw_polarization: kq_host entry out of range");
  if (d.k_list_host) {
    if (d.n_k_list < 1) return fail(GW_ERR_INVALID_ARG, "gw_polarization: n_k_list must be >= 1");
    for (int i = 0; i < d.n_k_list; ++i)
      if (d.k_list_host[i] < 0 || d.k_list_host[i] >= d.n_k)
        return fail(GW_ERR_INVALID_ARG, "gw_polarization: k_list_host entry out of range");
  }
  if (d.n_nodes < 0) return fail(GW_ERR_INVALID_ARG, "gw_polarization: n_nodes < 0");
  if (d.n_nodes > 0) {
    if (d.n_nodes < 2 || d.n_nodes > kMaxSlots)
      return fail(GW_ERR_INVALID_ARG, "gw_polarization: the spectral route needs 2..256 nodes");
    if (d.precision == GW_SPLIT_FP16 && d.n_nodes > kMaxOmega)
      return fail(GW_ERR_UNSUPPORTED, "gw_polarization: at most 64 nodes with GW_SPLIT_FP16");
    if (!d.nodes_host) return fail(GW_ERR_INVALID_ARG, "gw_polarization: nodes_host is NULL");
    for (int b = 0; b < d.n_nodes; ++b)
      if (!std::isfinite(d.nodes_host[b]) || d.nodes_host[b] <= 0.0 || (b > 0 && d.nodes_host[b] <= d.nodes_host[b - 1]))
        return fail(GW_ERR_INVALID_ARG, "gw_polarization: nodes must be finite, > 0 and increasing");
  }
  // Insulator: every summed occupied level below every summed unoccupied level at k+q.
  const int nb = d.n_occ + d.n_unocc;
  const int nk = d.k_list_host ? d.n_k_list : d.n_k;
  for (int i = 0; i < nk; ++i) {
    int k = d.k_list_host ? d.k_list_host[i] : i;
    int kq = d.kq_host ? d.kq_host[k] : (k + 1) % d.n_k;
    double hi = -INFINITY, lo = INFINITY;
    for (int n = d.occ_begin; n < d.occ_end; ++n) {
      double e = d.eps_host[(size_t)k * nb + n];
      if (!std::isfinite(e)) return fail(GW_ERR_INVALID_ARG, "gw_polarization: non-finite band energy");
      hi = std::max(hi, e);
    }
    for (int u = d.unocc_begin; u < d.unocc_end; ++u) {
      double e = d.eps_host[(size_t)kq * nb + d.n_occ + u];
      if (!std::isfinite(e)) return fail(GW_ERR_INVALID_ARG, "gw_polarization: non-finite band energy");
      lo = std::min(lo, e);
    }
    if (!(hi < lo)) {
      char buf[160];
      snprintf(buf, sizeof buf,
               "gw_polarization: k=%d: occupied level %.6g is not below unoccupied level %.6g at k+q "
               "(only insulators are supported)",
               k, hi, lo);
      return fail(GW_ERR_INVALID_ARG, buf);
    }
    if (d.n_nodes > 0) {
      // transition energies of this k lie in [lo - hi, top - bottom]
      double bottom = INFINITY, top = -INFINITY;
      for (int n = d.occ_begin; n < d.occ_end; ++n) bottom = std::min(bottom, d.eps_host[(size_t)k * nb + n]);
      for (int u = d.unocc_begin; u < d.unocc_end; ++u) top = std::max(top, d.eps_host[(size_t)kq * nb + d.n_occ + u]);
      if (lo - hi < d.nodes_host[0] || top - bottom > d.nodes_host[d.n_nodes - 1]) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "gw_polarization: k=%d: transition energies [%.6g, %.6g] are not inside the nodes [%.6g, %.6g]", k,
                 lo - hi, top - bottom, d.nodes_host[0], d.nodes_host[d.n_nodes - 1]);
        return fail(GW_ERR_INVALID_ARG, buf);
      }
    }
  }
  return GW_OK;
}

// One pass of the direct sum into the slots of d (frequencies, or the nodes of
// the spectral route when hat = 1); validated arguments, sized workspace.
int polarization_pass(hipStream_t s, const gw_pol_desc& d, int hat, void* ws) {
  int st;
  Plan pl = make_plan_direct(d);
  OmegaList om;
  om.n = d.n_omega;
  om.hat = hat;
  for (int j = 0; j < kMaxSlots; ++j) om.w[j] = j < d.n_omega ? d.omega_host[j] : 0.0;
  const int nb = d.n_occ + d.n_unocc;
  const size_t NN = (size_t)d.N * d.N;
  double2* P = reinterpret_cast<double2*>(d.P);
  if (!d.accumulate) {
    st = launch_fill_zero(s, d.P, NN * 2 * d.n_omega);
    if (st != GW_OK) return st;
  }
  std::vector<Chunk> chunks;
  const int nk = d.k_list_host ? d.n_k_list : d.n_k;
  for (int i = 0; i < nk; ++i) {
    int k = d.k_list_host ? d.k_list_host[i] : i;
    int kq = d.kq_host ? d.kq_host[k] : (k + 1) % d.n_k;
    const int nu = d.unocc_end - d.unocc_begin;
    const long total = (long)(d.occ_end - d.occ_begin) * nu;
    for (long tb = 0; tb < total; tb += pl.tc) {
      Chunk c;
      c.k = k;
      c.kq = kq;
      c.n0 = d.occ_begin;
      c.u0 = d.unocc_begin;
      c.nu = nu;
      c.tb = tb;
      c.T = (int)std::min<long>(pl.tc, total - tb);
      chunks.push_back(c);
    }
  }
  if (d.precision == GW_FP64) {
    Carver cv(ws);
    double2* M = cv.take<double2>((size_t)d.N * pl.tc);
    double* w = cv.take<double>((size_t)d.n_omega * pl.tc);
    const double2* U = static_cast<const double2*>(d.U);
    const double2* psi = static_cast<const double2*>(d.psi);
    for (const Chunk& c : chunks) {
      const double2* po = psi + ((size_t)c.k * nb + c.n0) * d.R;
      const double2* pu = psi + ((size_t)c.kq * nb + d.n_occ + c.u0) * d.R;
      if ((st = launch_weights_f64(s, d.eps, nb, d.n_occ, c, om, w)) != GW_OK) return st;
      if ((st = launch_project_f64(s, d.N, d.R, U, po, pu, c.nu, c.tb, c.T, M, c.T)) != GW_OK) return st;
      if ((st = launch_herk_f64(s, d.N, c.pairs(), M, c.pairs(), w, d.n_omega, P)) != GW_OK) return st;
    }
  } else {
    st = d.real_inputs ? tiled_polarization_real(s, d, chunks, pl.tc, om, ws)
                       : mfma_polarization(s, d, chunks, pl.tc, om, ws);
    if (st != GW_OK) return st;
  }
  return launch_hermitian_mirror(s, d.N, d.n_omega, P);
}
}  // namespace
}  // namespace gw

using namespace gw;

extern "C" {

const char* gw_last_error(void) { return g_last_error.c_str(); }

int gw_version(void) { return 100; }

int gw_project_workspace_size(int precision, int N, int R, int n_occ, int n_unocc, size_t* bytes) {
  if (!bytes) return fail(GW_ERR_INVALID_ARG, "gw_project_workspace_size: bytes_host is NULL");
  if (!valid_precision(precision)) return fail(GW_ERR_INVALID_ARG, "gw_project: unknown precision");
  if (N < 1 || R < 1 || n_occ < 1 || n_unocc < 1)
    return fail(GW_ERR_INVALID_ARG, "gw_project: sizes must be >= 1");
  *bytes = precision == GW_FP64 ? 0 : mfma_project_workspace(precision, N, R, n_occ, n_unocc);
  return GW_OK;
}

int gw_project(void* stream, int precision, int N, int R, int n_occ, int n_unocc, const void* U,
               const void* psi_occ, const void* psi_unocc, void* M, void* ws, size_t ws_bytes) {
  size_t need = 0;
  int st = gw_project_workspace_size(precision, N, R, n_occ, n_unocc, &need);
  if (st != GW_OK) return st;
  if (!U || !psi_occ || !psi_unocc || !M)
    return fail(GW_ERR_INVALID_ARG, "gw_project: null pointer among U, psi_occ, psi_unocc, M");
  if (need > 0 && (!ws || ws_bytes < need)) {
    return fail(GW_ERR_WORKSPACE, "gw_project: workspace smaller than gw_project_workspace_size");
  }
  if ((long long)n_occ * n_unocc > (1LL << 31)) return fail(GW_ERR_UNSUPPORTED, "gw_project: too many pairs");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == GW_FP64)
    return launch_project_f64(s, N, R, static_cast<const double2*>(U), static_cast<const double2*>(psi_occ),
                              static_cast<const double2*>(psi_unocc), n_unocc, 0, n_occ * n_unocc,
                              static_cast<double2*>(M), (long)n_occ * n_unocc);
  return mfma_project(s, precision, N, R, n_occ, n_unocc, U, psi_occ, psi_unocc, M, ws, ws_bytes);
}

int gw_polarization_workspace_size(const gw_pol_desc* d, size_t* bytes) {
  if (!bytes) return fail(GW_ERR_INVALID_ARG, "gw_polarization_workspace_size: bytes_host is NULL");
  if (!d) return fail(GW_ERR_INVALID_ARG, "gw_polarization_workspace_size: desc is NULL");
  if (!valid_precision(d->precision)) return fail(GW_ERR_INVALID_ARG, "gw_polarization: unknown precision");
  if (d->N < 1 || d->R < 1 || d->n_omega < 1 || d->occ_end <= d->occ_begin || d->unocc_end <= d->unocc_begin)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization_workspace_size: bad sizes or band ranges");
  if (d->chunk_pairs < 0) return fail(GW_ERR_INVALID_ARG, "gw_polarization: chunk_pairs < 0");
  if (d->real_inputs != 0 && d->real_inputs != 1)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization: real_inputs must be 0 or 1");
  if (d->real_inputs && d->precision != GW_SPLIT_BF16)
    return fail(GW_ERR_UNSUPPORTED, "gw_polarization: real inputs are supported with GW_SPLIT_BF16 only");
  if (d->n_nodes < 0 || d->n_nodes == 1 || d->n_nodes > kMaxSlots)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization: the spectral route needs 2..256 nodes");
  if (d->n_nodes > kMaxOmega && d->precision == GW_SPLIT_FP16)
    return fail(GW_ERR_UNSUPPORTED, "gw_polarization: at most 64 nodes with GW_SPLIT_FP16");
  *bytes = make_plan(*d).ws;
  return GW_OK;
}

int gw_polarization(void* stream, const gw_pol_desc* dp, void* ws, size_t ws_bytes) {
  int st = validate_desc(dp);
  if (st != GW_OK) return st;
  const gw_pol_desc& d = *dp;
  Plan pl = make_plan(d);
  if (!ws || ws_bytes < pl.ws) {
    char buf[128];
    snprintf(buf, sizeof buf, "gw_polarization: workspace of %zu bytes needed, %zu given", pl.ws, ws_bytes);
    return fail(GW_ERR_WORKSPACE, buf);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (d.n_nodes == 0) return polarization_pass(s, d, 0, ws);
  // spectral route: node matrices first (workspace head), then their transform
  double2* S = static_cast<double2*>(ws);
  const gw_pol_desc in = spectral_inner(d, S);
  if ((st = polarization_pass(s, in, 1, static_cast<char*>(ws) + node_bytes(d))) != GW_OK) return st;
  OmegaList nodes;
  nodes.n = d.n_nodes;
  nodes.hat = 1;
  for (int b = 0; b < kMaxSlots; ++b) nodes.w[b] = b < d.n_nodes ? d.nodes_host[b] : 0.0;
  return launch_spectral_combine(s, d.N, nodes, d.n_omega, d.omega_host, S, reinterpret_cast<double2*>(d.P),
                                 d.accumulate);
}

int gw_screen_workspace_size(int N, int n_omega, size_t* bytes) {
  if (!bytes) return fail(GW_ERR_INVALID_ARG, "gw_screen_workspace_size: bytes_host is NULL");
  if (N < 1 || n_omega < 1) return fail(GW_ERR_INVALID_ARG, "gw_screen: N and n_omega must be >= 1");
  *bytes = screen_workspace_bytes(N, n_omega);
  return GW_OK;
}

int gw_screen(void* stream, int N, int n_omega, const double* P, const double* v, double* W, int* info,
              void* ws, size_t ws_bytes) {
  size_t need = 0;
  int st = gw_screen_workspace_size(N, n_omega, &need);
  if (st != GW_OK) return st;
  if (!P || !v || !W || !info) return fail(GW_ERR_INVALID_ARG, "gw_screen: null pointer among P, v, W, info");
  if (P == W) return fail(GW_ERR_INVALID_ARG, "gw_screen: W may not alias P");
  if ((long long)N * N > (1LL << 31)) return fail(GW_ERR_UNSUPPORTED, "gw_screen: N too large");
  if (!ws || ws_bytes < need) return fail(GW_ERR_WORKSPACE, "gw_screen: workspace smaller than required");
  return screen_run(static_cast<hipStream_t>(stream), N, n_omega, reinterpret_cast<const double2*>(P), v,
                    reinterpret_cast<double2*>(W), info, ws);
}

}  // extern "C"
