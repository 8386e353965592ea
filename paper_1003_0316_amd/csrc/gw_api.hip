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

bool valid_precision(int p) { return p >= GW_FP64 && p <= GW_FP16; }
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

// Workspace of one call: the pass (and the spectral route's node matrices),
// then a device flag for the optional finite checks.
Plan make_plan(const gw_pol_desc& d) {
  Plan pl;
  if (d.n_nodes > 0) {
    pl = make_plan_direct(spectral_inner(d, nullptr));
    pl.ws += node_bytes(d);
  } else {
    pl = make_plan_direct(d);
  }
  pl.ws += kFlagBytes;
  return pl;
}

unsigned* flag_at_end(void* ws, size_t ws_need) {
  return reinterpret_cast<unsigned*>(static_cast<char*>(ws) + ws_need - kFlagBytes);
}

// GW_CHECK_FINITE on the inputs of a polarization call (one synchronisation).
int check_pol_inputs(hipStream_t s, const gw_pol_desc& d, unsigned* flag, const char* who) {
  const bool f64 = d.precision == GW_FP64;
  const size_t per = d.real_inputs ? 1 : 2;
  const size_t nb = (size_t)d.n_occ + d.n_unocc;
  int st;
  if ((st = launch_flag_clear(s, flag)) != GW_OK) return st;
  if ((st = launch_nonfinite(s, d.U, (size_t)d.N * d.R * per, f64, flag)) != GW_OK) return st;
  if ((st = launch_nonfinite(s, d.psi, (size_t)d.n_k * nb * d.R * per, f64, flag)) != GW_OK) return st;
  if ((st = launch_nonfinite(s, d.eps, (size_t)d.n_k * nb, true, flag)) != GW_OK) return st;
  unsigned h = 0;
  if ((st = read_flag(s, flag, &h)) != GW_OK) return st;
  if (h) return fail(GW_ERR_NONFINITE, std::string(who) + ": U, psi or eps holds Inf or NaN (nothing computed)");
  return GW_OK;
}

// GW_CHECK_FINITE on a result of n_doubles doubles (one synchronisation).
int check_result(hipStream_t s, const double* x, size_t n_doubles, unsigned* flag, const char* what) {
  int st;
  if ((st = launch_flag_clear(s, flag)) != GW_OK) return st;
  if ((st = launch_nonfinite(s, x, n_doubles, true, flag)) != GW_OK) return st;
  unsigned h = 0;
  if ((st = read_flag(s, flag, &h)) != GW_OK) return st;
  if (h) return fail(GW_ERR_NONFINITE, std::string(what) + " holds Inf or NaN");
  return GW_OK;
}

Plan make_plan_direct(const gw_pol_desc& d) {
  Plan pl;
  const long total = (long)(d.occ_end - d.occ_begin) * (d.unocc_end - d.unocc_begin);
  pl.tc = (int)std::max(1L, std::min<long>(default_chunk_pairs(d), total));
  if (d.precision == GW_FP64) {
    pl.ws = align_up((size_t)d.N * pl.tc * 16) + align_up((size_t)d.n_omega * pl.tc * sizeof(double));
  } else {
    pl.ws = d.real_inputs ? tiled_pol_workspace_real(d.N, d.R, pl.tc, d.n_omega)
                          : mfma_pol_workspace(d.precision, d.N, d.R, pl.tc, d.n_omega,
                                               (size_t)d.n_k * (d.n_occ + d.n_unocc));
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
  if (d.flags & ~GW_CHECK_FINITE) return fail(GW_ERR_INVALID_ARG, "gw_polarization: unknown flags");
  if (d.n_nodes < 0) return fail(GW_ERR_INVALID_ARG, "gw_polarization: n_nodes < 0");
  if (d.n_nodes > 0) {
    if (d.n_nodes < 2 || d.n_nodes > kMaxSlots)
      return fail(GW_ERR_INVALID_ARG, "gw_polarization: the spectral route needs 2..256 nodes");
    if ((d.precision == GW_SPLIT_FP16 || d.precision == GW_FP16) && d.n_nodes > kMaxOmega)
      return fail(GW_ERR_UNSUPPORTED, "gw_polarization: at most 64 nodes with the FP16 precisions");
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

// ---- learned path (gw_polarization_learned) --------------------------------------
int validate_learned(const gw_pol_desc* dp, const gw_learned_desc* l) {
  int st = validate_desc(dp);
  if (st != GW_OK) return st;
  const gw_pol_desc& d = *dp;
  if (!l || !l->mlp) return fail(GW_ERR_INVALID_ARG, "gw_polarization_learned: learned desc or its mlp is NULL");
  if (d.occ_begin != 0 || d.occ_end != d.n_occ || d.unocc_begin != 0 || d.unocc_end != d.n_unocc)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization_learned: the desc must cover every band (the cutoff is in the "
                                    "learned desc)");
  if (d.k_list_host || d.accumulate || d.n_nodes || d.real_inputs)
    return fail(GW_ERR_UNSUPPORTED, "gw_polarization_learned: needs all k-points, accumulate 0, the direct sum and "
                                    "complex inputs");
  if (d.n_k > 64) return fail(GW_ERR_UNSUPPORTED, "gw_polarization_learned: at most 64 k-sets");
  if (l->cut < 1 || l->cut >= d.n_unocc)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization_learned: need 1 <= cut < n_unocc");
  const gw_mlp& m = *l->mlp;
  auto ok_dim = [](int x) { return x == 32 || x == 64 || x == 128 || x == 256; };
  if (!ok_dim(m.n_in) || !ok_dim(m.width) || !ok_dim(m.n_out) || !m.wt)
    return fail(GW_ERR_INVALID_ARG, "gw_polarization_learned: perceptron sizes must be 32, 64, 128 or 256 and wt set");
  if (l->judge != 0 && l->judge != 1) return fail(GW_ERR_INVALID_ARG, "gw_polarization_learned: judge is 0 or 1");
  if (l->judge) {
    if (l->n_sample_occ < 1 || l->n_sample_occ > d.n_occ || d.n_k * l->n_sample_occ > 64)
      return fail(GW_ERR_INVALID_ARG,
                  "gw_polarization_learned: need 1 <= n_sample_occ <= n_occ and n_k * n_sample_occ <= 64");
    if (!std::isfinite(l->judge_tol) || l->judge_tol < 0.0)
      return fail(GW_ERR_INVALID_ARG, "gw_polarization_learned: judge_tol must be finite and >= 0");
  }
  return GW_OK;
}

// Workspace layout of a learned call: one polarization-pass region (the larger
// of the explicit and the fallback pass), the perceptron's rows, the surrogate
// kernels' scratch, the judge's projections and partial traces, the errors and
// the finite-check flag.
struct LearnedLayout {
  size_t pol, x, y, act, sws, mproj, pws, pws_bytes, part, err, total;
  int nu, parts_row;
};

LearnedLayout learned_layout(const gw_pol_desc& d, const gw_learned_desc& l) {
  LearnedLayout L{};
  gw_pol_desc a = d;
  a.unocc_end = l.cut;
  gw_pol_desc b = d;
  b.unocc_begin = l.cut;
  b.accumulate = 1;
  const size_t pol = std::max(make_plan_direct(a).ws, make_plan_direct(b).ws);
  const size_t rows = (size_t)d.n_omega * d.N;
  gw_surr_desc sd{};
  sd.N = d.N;
  sd.n_omega = d.n_omega;
  sd.n_k = d.n_k;
  sd.n_occ = d.n_occ;
  sd.n_unocc = d.n_unocc;
  sd.cut = l.cut;
  sd.n_in = l.mlp->n_in;
  sd.eps = d.eps;
  sd.P_ret = d.P;
  size_t sws = 0;
  gw_surrogate_workspace_size(&sd, &sws);
  L.nu = d.n_unocc - l.cut;
  L.parts_row = sample_trace_parts(d.N, L.nu);
  const int n_rows = l.judge ? d.n_k * l.n_sample_occ : 0;
  const size_t mproj = l.judge ? (size_t)d.N * L.nu * cplx_bytes(d.precision) : 0;
  const size_t pws = (l.judge && d.precision != GW_FP64)
                         ? mfma_project_workspace(d.precision, d.N, d.R, 1, L.nu) : 0;
  Carver cv(nullptr);
  L.pol = cv.off; cv.take<char>(pol);
  L.x = cv.off; cv.take<float>(rows * l.mlp->n_in);
  L.y = cv.off; cv.take<float>(rows * l.mlp->n_out);
  L.act = cv.off; cv.take<float>(rows * 4 * (size_t)l.mlp->width);
  L.sws = cv.off; cv.take<char>(sws);
  L.mproj = cv.off; cv.take<char>(mproj);
  L.pws = cv.off; cv.take<char>(pws);
  L.pws_bytes = pws;
  L.part = cv.off; cv.take<double>((size_t)std::max(1, n_rows) * L.parts_row * d.n_omega);
  L.err = cv.off; cv.take<double>(kMaxOmega);
  cv.take<char>(kFlagBytes);
  L.total = cv.off;
  return L;
}

// Occupied band of judge sample i of n: evenly from the lowest (0) to the
// highest (n_occ - 1); the middle band when n = 1.
int sample_band(int i, int n, int n_occ) {
  if (n == 1) return n_occ / 2;
  return (int)(((long)i * (n_occ - 1) + (n - 1) / 2) / (n - 1));
}

int polarization_learned(hipStream_t s, const gw_pol_desc& d, const gw_learned_desc& l, char* ws,
                         const LearnedLayout& L) {
  int st;
  unsigned* flag = reinterpret_cast<unsigned*>(ws + L.total - kFlagBytes);
  const bool check = d.flags & GW_CHECK_FINITE;
  if (check && (st = check_pol_inputs(s, d, flag, "gw_polarization_learned")) != GW_OK) return st;
  // 1. explicit bands [0, cut)
  gw_pol_desc a = d;
  a.unocc_end = l.cut;
  if ((st = polarization_pass(s, a, 0, ws + L.pol)) != GW_OK) return st;
  // 2. features and the perceptron
  gw_surr_desc sd{};
  sd.N = d.N;
  sd.n_omega = d.n_omega;
  sd.omega_host = d.omega_host;
  sd.n_k = d.n_k;
  sd.n_occ = d.n_occ;
  sd.n_unocc = d.n_unocc;
  sd.cut = l.cut;
  sd.kq_host = d.kq_host;
  sd.eps = d.eps;
  sd.P_ret = d.P;
  sd.n_in = l.mlp->n_in;
  size_t sws = 0;
  if ((st = gw_surrogate_workspace_size(&sd, &sws)) != GW_OK) return st;
  float* X = reinterpret_cast<float*>(ws + L.x);
  float* Y = reinterpret_cast<float*>(ws + L.y);
  float* act = reinterpret_cast<float*>(ws + L.act);
  const int rows = d.n_omega * d.N;
  if ((st = gw_surrogate_features(s, &sd, X, ws + L.sws, sws)) != GW_OK) return st;
  if ((st = gw_mlp_forward(s, l.mlp, X, rows, Y, act)) != GW_OK) return st;
  // 3. judge on an explicit sample of the left-out bands
  bool fallback = false;
  if (l.judge) {
    OmegaList om;
    om.n = d.n_omega;
    om.hat = 0;
    for (int j = 0; j < kMaxSlots; ++j) om.w[j] = j < d.n_omega ? d.omega_host[j] : 0.0;
    const int nb = d.n_occ + d.n_unocc;
    const size_t eb = cplx_bytes(d.precision);
    const char* psi = static_cast<const char*>(d.psi);
    double* part = reinterpret_cast<double*>(ws + L.part);
    int rk[64], ro[64];
    int n_rows = 0;
    for (int k = 0; k < d.n_k; ++k) {
      const int kq = d.kq_host ? d.kq_host[k] : (k + 1) % d.n_k;
      for (int i = 0; i < l.n_sample_occ; ++i) {
        const int n = sample_band(i, l.n_sample_occ, d.n_occ);
        const void* po = psi + ((size_t)k * nb + n) * d.R * eb;
        const void* pu = psi + ((size_t)kq * nb + d.n_occ + l.cut) * d.R * eb;
        void* M = ws + L.mproj;
        if (d.precision == GW_FP64) {
          st = launch_project_f64(s, d.N, d.R, static_cast<const double2*>(d.U), static_cast<const double2*>(po),
                                  static_cast<const double2*>(pu), L.nu, 0, L.nu, static_cast<double2*>(M), L.nu);
        } else {
          st = mfma_project(s, d.precision, d.N, d.R, 1, L.nu, d.U, po, pu, M, ws + L.pws, L.pws_bytes);
        }
        if (st != GW_OK) return st;
        if ((st = launch_sample_trace(s, d.precision == GW_FP64, M, d.N, L.nu, L.nu, d.eps + (size_t)k * nb + n,
                                      d.eps + (size_t)kq * nb + d.n_occ + l.cut, om,
                                      part + (size_t)n_rows * L.parts_row * d.n_omega)) != GW_OK)
          return st;
        rk[n_rows] = k;
        ro[n_rows] = n;
        ++n_rows;
      }
    }
    double* err = reinterpret_cast<double*>(ws + L.err);
    if ((st = surrogate_judge_traces(s, sd, Y, l.mlp->n_out, part, n_rows * L.parts_row, n_rows, rk, ro, err,
                                     ws + L.sws)) != GW_OK)
      return st;
    double eh[kMaxOmega];
    GW_HIP(hipMemcpyAsync(eh, err, d.n_omega * sizeof(double), hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < d.n_omega; ++j) {
      if (!(eh[j] <= l.judge_tol)) fallback = true;   // also for NaN
      if (l.judge_err_host) l.judge_err_host[j] = eh[j];
    }
  }
  if (l.used_fallback_host) *l.used_fallback_host = fallback ? 1 : 0;
  // 4. the correction, or the explicit left-out bands
  if (!fallback) {
    if ((st = gw_surrogate_apply(s, d.N, d.n_omega, Y, l.mlp->n_out, d.P)) != GW_OK) return st;
  } else {
    gw_pol_desc b = d;
    b.unocc_begin = l.cut;
    b.accumulate = 1;
    if ((st = polarization_pass(s, b, 0, ws + L.pol)) != GW_OK) return st;
  }
  if (check) return check_result(s, d.P, (size_t)d.n_omega * d.N * d.N * 2, flag,
                                 "gw_polarization_learned: the result P");
  return GW_OK;
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
  if (d->n_nodes > kMaxOmega && (d->precision == GW_SPLIT_FP16 || d->precision == GW_FP16))
    return fail(GW_ERR_UNSUPPORTED, "gw_polarization: at most 64 nodes with the FP16 precisions");
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
  unsigned* flag = flag_at_end(ws, pl.ws);
  const bool check = d.flags & GW_CHECK_FINITE;
  if (check && (st = check_pol_inputs(s, d, flag, "gw_polarization")) != GW_OK) return st;
  if (d.n_nodes == 0) {
    if ((st = polarization_pass(s, d, 0, ws)) != GW_OK) return st;
  } else {
    // spectral route: node matrices first (workspace head), then their transform
    double2* S = static_cast<double2*>(ws);
    const gw_pol_desc in = spectral_inner(d, S);
    if ((st = polarization_pass(s, in, 1, static_cast<char*>(ws) + node_bytes(d))) != GW_OK) return st;
    OmegaList nodes;
    nodes.n = d.n_nodes;
    nodes.hat = 1;
    for (int b = 0; b < kMaxSlots; ++b) nodes.w[b] = b < d.n_nodes ? d.nodes_host[b] : 0.0;
    if ((st = launch_spectral_combine(s, d.N, nodes, d.n_omega, d.omega_host, S, reinterpret_cast<double2*>(d.P),
                                      d.accumulate)) != GW_OK)
      return st;
  }
  if (check) return check_result(s, d.P, (size_t)d.n_omega * d.N * d.N * 2, flag, "gw_polarization: the result P");
  return GW_OK;
}

int gw_polarization_learned_workspace_size(const gw_pol_desc* d, const gw_learned_desc* l, size_t* bytes) {
  if (!bytes) return fail(GW_ERR_INVALID_ARG, "gw_polarization_learned_workspace_size: bytes_host is NULL");
  int st = validate_learned(d, l);
  if (st != GW_OK) return st;
  *bytes = learned_layout(*d, *l).total;
  return GW_OK;
}

int gw_polarization_learned(void* stream, const gw_pol_desc* d, const gw_learned_desc* l, void* ws,
                            size_t ws_bytes) {
  int st = validate_learned(d, l);
  if (st != GW_OK) return st;
  const LearnedLayout L = learned_layout(*d, *l);
  if (!ws || ws_bytes < L.total) {
    char buf[160];
    snprintf(buf, sizeof buf, "gw_polarization_learned: workspace of %zu bytes needed, %zu given", L.total,
             ws_bytes);
    return fail(GW_ERR_WORKSPACE, buf);
  }
  return polarization_learned(static_cast<hipStream_t>(stream), *d, *l, static_cast<char*>(ws), L);
}

int gw_screen_workspace_size(int N, int n_omega, size_t* bytes) {
  if (!bytes) return fail(GW_ERR_INVALID_ARG, "gw_screen_workspace_size: bytes_host is NULL");
  if (N < 1 || n_omega < 1) return fail(GW_ERR_INVALID_ARG, "gw_screen: N and n_omega must be >= 1");
  *bytes = screen_workspace_bytes(N, n_omega) + kFlagBytes;
  return GW_OK;
}

int gw_screen_ex(void* stream, int N, int n_omega, const double* P, const double* v, double* W, int* info,
                 int flags, void* ws, size_t ws_bytes) {
  size_t need = 0;
  int st = gw_screen_workspace_size(N, n_omega, &need);
  if (st != GW_OK) return st;
  if (!P || !v || !W || !info) return fail(GW_ERR_INVALID_ARG, "gw_screen: null pointer among P, v, W, info");
  if (P == W) return fail(GW_ERR_INVALID_ARG, "gw_screen: W may not alias P");
  if (flags & ~(GW_CHECK_FINITE | GW_CHECK_HPD)) return fail(GW_ERR_INVALID_ARG, "gw_screen: unknown flags");
  if ((long long)N * N > (1LL << 31)) return fail(GW_ERR_UNSUPPORTED, "gw_screen: N too large");
  if (!ws || ws_bytes < need) return fail(GW_ERR_WORKSPACE, "gw_screen: workspace smaller than required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* flag = flag_at_end(ws, need);
  if (flags & GW_CHECK_FINITE) {
    if ((st = launch_flag_clear(s, flag)) != GW_OK) return st;
    if ((st = launch_nonfinite(s, P, (size_t)n_omega * N * N * 2, true, flag)) != GW_OK) return st;
    if ((st = launch_nonfinite(s, v, (size_t)N, true, flag)) != GW_OK) return st;
    unsigned h = 0;
    if ((st = read_flag(s, flag, &h)) != GW_OK) return st;
    if (h) return fail(GW_ERR_NONFINITE, "gw_screen: P or v holds Inf or NaN (nothing computed)");
  }
  if ((st = screen_run(s, N, n_omega, reinterpret_cast<const double2*>(P), v, reinterpret_cast<double2*>(W), info,
                       ws)) != GW_OK)
    return st;
  if (flags & GW_CHECK_HPD) {
    int ih[kMaxSlots];
    int first = -1, col = 0;
    for (int j0 = 0; j0 < n_omega; j0 += kMaxSlots) {
      const int nj = std::min(kMaxSlots, n_omega - j0);
      GW_HIP(hipMemcpyAsync(ih, info + j0, nj * sizeof(int), hipMemcpyDeviceToHost, s));
      GW_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < nj && first < 0; ++j)
        if (ih[j] != 0) {
          first = j0 + j;
          col = ih[j] - 1;
        }
    }
    if (first >= 0) {
      char buf[200];
      snprintf(buf, sizeof buf,
               "gw_screen: eps = 1 - sqrt(v) P sqrt(v) is not positive definite at frequency %d (pivot column %d; "
               "info holds every frequency's column)",
               first, col);
      return fail(GW_ERR_NOT_HPD, buf);
    }
  }
  if (flags & GW_CHECK_FINITE) return check_result(s, W, (size_t)n_omega * N * N * 2, flag, "gw_screen: the result W");
  return GW_OK;
}

int gw_screen(void* stream, int N, int n_omega, const double* P, const double* v, double* W, int* info,
              void* ws, size_t ws_bytes) {
  return gw_screen_ex(stream, N, n_omega, P, v, W, info, 0, ws, ws_bytes);
}

}  // extern "C"
