// Correlation self-energy on the imaginary axis (Eq. SEc_AC): diagonal
// elements Sigma_c^n(i w) for a list of states, summed over the momentum
// transfers t and all bands n' of the set (s + t) mod N_k:
//
//   Sigma_c^n(i w) = -(1/2pi) sum_t sum_n' sum_j  w_j(w, e_n' - mu)  q_j^{t n n'}
//   q_j = m^H (W_j - diag v) m,   m_I = sum_r U_Ir conj(psi_n(r)) psi_n'(r)
//
// with w_j the weights of the frequency integral over the interpolant of
// W^c between the imaginary mesh points: a clamped cubic spline in
// lambda = w / (1 + w) (slope 0 at w = 0, where W is even; at the last point
// the slope of the w^-2 tail) continued by q_L (w_L / w')^2, integrated
// stepwise in closed form.  The weights and the final sums run in FP64; the
// quadratic forms in FP64 or on the split-BF16 GEMM core.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "gw_internal.hpp"
#include "gw_mfma.hpp"

namespace gw {
namespace {

constexpr int kMaxMesh = 64;
struct Mesh {
  int n;
  double w[kMaxMesh];
};

// ------------------------------------------------------------ complex FP64
struct cd {
  double x, y;
};
__device__ inline cd mk(double x, double y) { return cd{x, y}; }
__device__ inline cd add(cd a, cd b) { return mk(a.x + b.x, a.y + b.y); }
__device__ inline cd sub(cd a, cd b) { return mk(a.x - b.x, a.y - b.y); }
__device__ inline cd mul(cd a, cd b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline cd scl(cd a, double s) { return mk(a.x * s, a.y * s); }
__device__ inline cd dvd(cd a, cd b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return mk((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return mk((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}
__device__ inline double cabs_(cd a) { return hypot(a.x, a.y); }
__device__ inline cd clog_(cd a) { return mk(log(cabs_(a)), atan2(a.y, a.x)); }
// principal arctangent, (i/2) [log(1 - i z) - log(1 + i z)]
__device__ inline cd catan_(cd z) {
  const cd iz = mk(-z.y, z.x);
  const cd d = sub(clog_(sub(mk(1.0, 0.0), iz)), clog_(add(mk(1.0, 0.0), iz)));
  return mk(-0.5 * d.y, 0.5 * d.x);
}

// int_0^h x^p / (x + d) dx: convergent series for |d| > 2h, else the
// recurrence F_p = h^p / p - d F_{p-1} from F_0 = log(1 + h/d).
__device__ inline cd int_pow_over_lin(int p, cd d, double h) {
  if (cabs_(d) > 2.0 * h) {
    const cd ratio = scl(dvd(mk(1.0, 0.0), d), -h);          // -h/d
    cd t = dvd(mk(pow(h, p + 1), 0.0), d);                     // h^(p+1)/d
    cd acc = mk(0.0, 0.0);
    for (int m = 0; m < 200; ++m) {
      const cd c = scl(t, 1.0 / (p + m + 1));
      acc = add(acc, c);
      if (cabs_(c) < 1e-18 * cabs_(acc)) break;
      t = mul(t, ratio);
    }
    return acc;
  }
  cd F = clog_(add(mk(1.0, 0.0), dvd(mk(h, 0.0), d)));
  for (int k = 1; k <= p; ++k) F = sub(mk(pow(h, k) / k, 0.0), mul(d, F));
  return F;
}

// ------------------------------------------------------------ spline basis
// Clamped cubic spline in lambda through unit data e_j (one thread per j):
// slopes m_i from C2 continuity (a tridiagonal system, Thomas algorithm),
// m_0 = 0, m_L = s_end q_L; Hermite coefficients per interval.
__global__ void spline_basis_kernel(Mesh mesh, double* __restrict__ C) {
  const int j = threadIdx.x;
  const int n = mesh.n, ni = n - 1;
  if (j >= n) return;
  double lam[kMaxMesh], q[kMaxMesh], m[kMaxMesh], cp[kMaxMesh], dp[kMaxMesh];
  for (int i = 0; i < n; ++i) {
    lam[i] = mesh.w[i] / (1.0 + mesh.w[i]);
    q[i] = i == j ? 1.0 : 0.0;
  }
  const double wl = mesh.w[n - 1], ll = lam[n - 1];
  m[0] = 0.0;
  m[n - 1] = -2.0 / wl / ((1.0 - ll) * (1.0 - ll)) * q[n - 1];
  // interior rows i = 1..n-2: h_i m_{i-1} + 2(h_{i-1} + h_i) m_i + h_{i-1} m_{i+1} = 3(h_i d_{i-1} + h_{i-1} d_i)
  for (int i = 1; i <= n - 2; ++i) {
    const double hm = lam[i] - lam[i - 1], hp = lam[i + 1] - lam[i];
    const double dm = (q[i] - q[i - 1]) / hm, dq = (q[i + 1] - q[i]) / hp;
    double a = hp, b = 2.0 * (hm + hp), c = hm, r = 3.0 * (hp * dm + hm * dq);
    if (i == 1) {
      r -= a * m[0];
      a = 0.0;
    }
    if (i == n - 2) {
      r -= c * m[n - 1];
      c = 0.0;
    }
    if (i == 1) {
      cp[i] = c / b;
      dp[i] = r / b;
    } else {
      const double den = b - a * cp[i - 1];
      cp[i] = c / den;
      dp[i] = (r - a * dp[i - 1]) / den;
    }
  }
  for (int i = n - 2; i >= 1; --i) m[i] = dp[i] - (i < n - 2 ? cp[i] * m[i + 1] : 0.0);
  for (int i = 0; i < ni; ++i) {
    const double h = lam[i + 1] - lam[i], dl = (q[i + 1] - q[i]) / h;
    double* c = C + (size_t)i * 4 * n;
    c[0 * n + j] = q[i];
    c[1 * n + j] = m[i];
    c[2 * n + j] = (3.0 * dl - 2.0 * m[i] - m[i + 1]) / h;
    c[3 * n + j] = (m[i] + m[i + 1] - 2.0 * dl) / (h * h);
  }
}

// w[b][o][j]: weight of mesh point j in int dw' q(i w') / (i w_o + i w' - e_b)
// over the spline-plus-tail interpolant, e_b = eps[b] - mu.  On interval i the
// folded kernel times dw'/dlambda is -i/(lambda + c1) + i/(lambda + c2) with
// a = i w - e, c1 = a / (i - a), c2 = a / (-i - a); the tail gives
// w_L^2 (2/a) [1/w_L - (1/a)((pi/2) sgn(-e) - atan(w_L / a))].
// One wavefront per (band b, output frequency o): its lanes first form the
// interval integrals J[i][p] = -i F_p(lambda_i + c1) + i F_p(lambda_i + c2)
// (shared by every mesh point j) in LDS, then lane j contracts them with the
// spline coefficients C[i][p][j].
__global__ __launch_bounds__(256) void sigma_weights_kernel(Mesh mesh, Mesh out, int nb,
                                                            const double* __restrict__ eps, double mu,
                                                            const double* __restrict__ C, double2* __restrict__ wts) {
  __shared__ cd Js[4][(kMaxMesh - 1) * 4];
  const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long item = blockIdx.x * 4L + g;
  const bool live = item < (long)nb * out.n;
  const int n = mesh.n, ni = n - 1;
  const int o = live ? (int)(item % out.n) : 0;
  const int b = live ? (int)(item / out.n) : 0;
  const double e = live ? eps[b] - mu : 1.0;
  const double w = out.w[o];
  const cd a = mk(-e, w);
  const cd c1 = dvd(a, sub(mk(0.0, 1.0), a));
  const cd c2 = dvd(a, sub(mk(0.0, -1.0), a));
  for (int q = lane; q < ni * 4; q += 64) {
    const int i = q >> 2, p = q & 3;
    const double l0 = mesh.w[i] / (1.0 + mesh.w[i]);
    const double l1 = mesh.w[i + 1] / (1.0 + mesh.w[i + 1]);
    const double h = l1 - l0;
    const cd f1 = int_pow_over_lin(p, add(mk(l0, 0.0), c1), h);
    const cd f2 = int_pow_over_lin(p, add(mk(l0, 0.0), c2), h);
    const cd df = sub(f2, f1);
    Js[g][q] = mk(-df.y, df.x);                                  // -i f1 + i f2
  }
  __syncthreads();
  if (!live || lane >= n) return;
  const int j = lane;
  cd acc = mk(0.0, 0.0);
  for (int q = 0; q < ni * 4; ++q) {
    const double coef = C[(size_t)q * n + j];
    if (coef != 0.0) acc = add(acc, scl(Js[g][q], coef));
  }
  if (j == n - 1) {
    const double wl = mesh.w[n - 1];
    const cd inv_a = dvd(mk(1.0, 0.0), a);
    const cd at = catan_(scl(inv_a, wl));
    const double sg = e < 0.0 ? 1.0 : -1.0;                    // sgn(-e)
    const cd inner = sub(mk(1.0 / wl, 0.0), mul(inv_a, sub(mk(0.5 * M_PI * sg, 0.0), at)));
    acc = add(acc, scl(mul(inv_a, inner), 2.0 * wl * wl));
  }
  wts[item * n + j] = make_double2(acc.x, acc.y);
}

// Y = (W - diag v) M: complex FP64, 64 x 64 output tiles, 256 threads with
// 4 x 4 outputs each, K stages of 16 through LDS.
__global__ __launch_bounds__(256) void zgemm_shift_kernel(int N, int nb, const double2* __restrict__ W,
                                                          const double* __restrict__ v,
                                                          const double2* __restrict__ M, double2* __restrict__ Y) {
  __shared__ double2 As[64][17];
  __shared__ double2 Bs[16][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < N; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int rr = e / 16, kk = e % 16;
      const int gr = r0 + rr, gk = k0 + kk;
      double2 x = make_double2(0.0, 0.0);
      if (gr < N && gk < N) {
        x = W[(size_t)gr * N + gk];
        if (gr == gk) x.x -= v[gr];
      }
      As[rr][kk] = x;
    }
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, cc = e % 64;
      const int gk = k0 + kk, gc = c0 + cc;
      Bs[kk][cc] = (gk < N && gc < nb) ? M[(size_t)gk * nb + gc] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[ty * 4 + i][kk];
#pragma unroll
      for (int i = 0; i < 4; ++i) b[i] = Bs[kk][tx * 4 + i];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          acc[i][l].x = fma(a[i].x, b[l].x, fma(-a[i].y, b[l].y, acc[i][l].x));
          acc[i][l].y = fma(a[i].x, b[l].y, fma(a[i].y, b[l].x, acc[i][l].y));
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int gr = r0 + ty * 4 + i, gc = c0 + tx * 4 + l;
      if (gr < N && gc < nb) Y[(size_t)gr * nb + gc] = acc[i][l];
    }
}

// q[n'] = Re sum_mu conj(M[mu][n']) Y[mu][n'] in two fixed-order passes (32
// columns x one chunk of rows per workgroup, then the chunks in order).
constexpr int CD_CHUNKS64 = 16;

__global__ __launch_bounds__(256) void coldot_f64_kernel(int N, int nb, const double2* __restrict__ M,
                                                         const double2* __restrict__ Y, int rows_per_chunk,
                                                         double* __restrict__ part) {
  __shared__ double red[8][32];
  const int cx = threadIdx.x & 31, ry = threadIdx.x >> 5;
  const int c = blockIdx.x * 32 + cx;
  const int r0 = blockIdx.y * rows_per_chunk, r1 = min(N, r0 + rows_per_chunk);
  double acc = 0.0;
  if (c < nb)
    for (int r = r0 + ry; r < r1; r += 8) {
      const double2 m = M[(size_t)r * nb + c], y = Y[(size_t)r * nb + c];
      acc = fma(m.x, y.x, fma(m.y, y.y, acc));
    }
  red[ry][cx] = acc;
  __syncthreads();
  if (ry == 0 && c < nb) {
    double t = red[0][cx];
#pragma unroll
    for (int g = 1; g < 8; ++g) t += red[g][cx];
    part[(size_t)blockIdx.y * nb + c] = t;
  }
}

__global__ void coldot_sum_kernel(int nb, int chunks, const double* __restrict__ part, double* __restrict__ q) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nb) return;
  double t = 0.0;
  for (int k = 0; k < chunks; ++k) t += part[(size_t)k * nb + c];
  q[c] = t;
}

// sigma[o] += -(1/2pi) sum_b sum_j w[b][o][j] q[j][b]; one block per output
// frequency, fixed-order reduction.
__global__ __launch_bounds__(256) void sigma_contract_kernel(int nb, int n_mesh, int n_out,
                                                             const double2* __restrict__ wts,
                                                             const double* __restrict__ q, long ldq,
                                                             double2* __restrict__ sig) {
  __shared__ double rx[256], ry[256];
  const int o = blockIdx.x;
  double ax = 0.0, ay = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    const double2* w = wts + ((size_t)b * n_out + o) * n_mesh;
    for (int j = 0; j < n_mesh; ++j) {
      const double qq = q[(size_t)j * ldq + b];
      ax = fma(w[j].x, qq, ax);
      ay = fma(w[j].y, qq, ay);
    }
  }
  rx[threadIdx.x] = ax;
  ry[threadIdx.x] = ay;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      rx[threadIdx.x] += rx[threadIdx.x + s];
      ry[threadIdx.x] += ry[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double f = -1.0 / (2.0 * M_PI);
    sig[o].x += f * rx[0];
    sig[o].y += f * ry[0];
  }
}

__global__ void zero_c128_kernel(double2* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

// ------------------------------------------------------------ host side
int validate_sigma(const gw_sigma_desc* dp) {
  if (!dp) return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: desc is NULL");
  const gw_sigma_desc& d = *dp;
  if (d.precision != GW_FP64 && d.precision != GW_SPLIT_BF16)
    return fail(GW_ERR_UNSUPPORTED, "gw_sigma_c: precision must be GW_FP64 or GW_SPLIT_BF16");
  if (d.n_k < 1 || d.N < 1 || d.R < 1 || d.n_bands < 1 || d.n_states < 1)
    return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: sizes must be >= 1");
  if (d.n_mesh < 2 || d.n_mesh > kMaxMesh || !d.mesh_host)
    return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: the mesh needs 2..64 points");
  if (d.mesh_host[0] != 0.0) return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: the mesh must start at 0");
  for (int j = 1; j < d.n_mesh; ++j)
    if (!std::isfinite(d.mesh_host[j]) || !(d.mesh_host[j] > d.mesh_host[j - 1]))
      return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: mesh points must be finite and increasing");
  if (d.n_out < 1 || d.n_out > kMaxMesh || !d.omega_out_host)
    return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: 1..64 output frequencies");
  for (int o = 0; o < d.n_out; ++o)
    if (!std::isfinite(d.omega_out_host[o]) || d.omega_out_host[o] < 0.0)
      return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: output frequencies must be finite and >= 0");
  if (!d.state_set_host || !d.state_band_host) return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: state lists are NULL");
  for (int i = 0; i < d.n_states; ++i)
    if (d.state_set_host[i] < 0 || d.state_set_host[i] >= d.n_k || d.state_band_host[i] < 0 ||
        d.state_band_host[i] >= d.n_bands)
      return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: state out of range");
  if (!std::isfinite(d.mu)) return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: mu must be finite");
  if (!d.eps_host || !d.eps || !d.U || !d.psi || !d.W_host || !d.v || !d.sigma)
    return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: NULL pointer");
  for (int t = 0; t < d.n_k; ++t)
    if (!d.W_host[t]) return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: W_host entry is NULL");
  for (size_t i = 0; i < (size_t)d.n_k * d.n_bands; ++i) {
    const double e = d.eps_host[i] - d.mu;
    if (!std::isfinite(e) || e == 0.0)
      return fail(GW_ERR_INVALID_ARG, "gw_sigma_c: band energies must be finite and differ from mu");
  }
  return GW_OK;
}

// States per batch of the split path (they share the W^c operand words of a
// transfer and one wide GEMM per mesh point).
constexpr int kSigmaBatch = 16;

struct SigmaWs {
  size_t total = 0;
  size_t quad = 0;   // split path: tiled operands
  int batch = 1;     // split path: states per batch
  long ldq = 0;      // columns of q
};

SigmaWs sigma_ws(const gw_sigma_desc& d) {
  SigmaWs w;
  const int ni = d.n_mesh - 1;
  if (d.precision == GW_FP64) {
    w.ldq = d.n_bands;
  } else {
    w.batch = std::min(d.n_states, kSigmaBatch);
    w.ldq = tiled_sigma_cols(d.n_bands, w.batch);
  }
  size_t t = align_up((size_t)ni * 4 * d.n_mesh * sizeof(double)) +
             align_up((size_t)d.n_k * d.n_bands * d.n_out * d.n_mesh * sizeof(double2)) +
             align_up((size_t)d.n_mesh * w.ldq * sizeof(double));
  if (d.precision == GW_FP64) {
    t += 2 * align_up((size_t)d.N * d.n_bands * sizeof(double2)) +
         align_up((size_t)CD_CHUNKS64 * d.n_bands * sizeof(double));
  } else {
    w.quad = tiled_sigma_workspace(d.N, d.R, d.n_bands, w.batch);
    t += align_up(w.quad);
  }
  w.total = t;
  return w;
}

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" int gw_sigma_c_workspace_size(const gw_sigma_desc* d, size_t* bytes) {
  if (!bytes) return fail(GW_ERR_INVALID_ARG, "gw_sigma_c_workspace_size: bytes is NULL");
  int st = validate_sigma(d);
  if (st != GW_OK) return st;
  *bytes = sigma_ws(*d).total;
  return GW_OK;
}

extern "C" int gw_sigma_c(void* stream, const gw_sigma_desc* dp, void* ws, size_t ws_bytes) {
  int st = validate_sigma(dp);
  if (st != GW_OK) return st;
  const gw_sigma_desc& d = *dp;
  const SigmaWs need = sigma_ws(d);
  if (!ws || ws_bytes < need.total) return fail(GW_ERR_WORKSPACE, "gw_sigma_c: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Mesh mesh{}, out{};
  mesh.n = d.n_mesh;
  for (int j = 0; j < d.n_mesh; ++j) mesh.w[j] = d.mesh_host[j];
  out.n = d.n_out;
  for (int o = 0; o < d.n_out; ++o) out.w[o] = d.omega_out_host[o];
  const int nb = d.n_bands, ni = d.n_mesh - 1;
  Carver cv(ws);
  double* C = cv.take<double>((size_t)ni * 4 * d.n_mesh);
  double2* wts = cv.take<double2>((size_t)d.n_k * nb * d.n_out * d.n_mesh);   // per band set
  double* q = cv.take<double>((size_t)d.n_mesh * need.ldq);
  double2* sig = static_cast<double2*>(d.sigma);
  hipLaunchKernelGGL(spline_basis_kernel, dim3(1), dim3(kMaxMesh), 0, s, mesh, C);
  GW_LAUNCHED("spline_basis_kernel");
  hipLaunchKernelGGL(zero_c128_kernel, dim3((d.n_states * d.n_out + 255) / 256), dim3(256), 0, s, sig,
                     d.n_states * d.n_out);
  GW_LAUNCHED("zero_c128_kernel");
  const long nw = (long)nb * d.n_out * d.n_mesh;
  const long nbo = (long)nb * d.n_out;
  // the weights depend on the band set only: once per set
  for (int k = 0; k < d.n_k; ++k) {
    ProfScope prof(s, "sigma_weights_kernel");
    hipLaunchKernelGGL(sigma_weights_kernel, dim3((unsigned)((nbo + 3) / 4)), dim3(256), 0, s, mesh, out, nb,
                       d.eps + (size_t)k * nb, d.mu, C, wts + (size_t)k * nw);
    GW_LAUNCHED("sigma_weights_kernel");
  }
  bool u_tiled = false;
  double2* M64 = nullptr;
  double2* Y64 = nullptr;
  double* part = nullptr;
  void* quad_ws = nullptr;
  if (d.precision == GW_FP64) {
    M64 = cv.take<double2>((size_t)d.N * nb);
    Y64 = cv.take<double2>((size_t)d.N * nb);
    part = cv.take<double>((size_t)CD_CHUNKS64 * nb);
  } else {
    quad_ws = cv.take<char>(need.quad);
  }
  if (d.precision == GW_FP64) {
    for (int si = 0; si < d.n_states; ++si) {
      const int s0 = d.state_set_host[si], n0 = d.state_band_host[si];
      for (int t = 0; t < d.n_k; ++t) {
        const int s2 = (s0 + t) % d.n_k;
        const double2* W = static_cast<const double2*>(d.W_host[t]);
        const double2* psi = static_cast<const double2*>(d.psi);
        const double2* pstate = psi + ((size_t)s0 * nb + n0) * d.R;
        const double2* pall = psi + (size_t)s2 * nb * d.R;
        if ((st = launch_project_f64(s, d.N, d.R, static_cast<const double2*>(d.U), pstate, pall, nb, 0, nb, M64,
                                     nb)) != GW_OK)
          return st;
        for (int j = 0; j < d.n_mesh; ++j) {
          {
            ProfScope prof(s, "zgemm_shift_kernel");
            hipLaunchKernelGGL(zgemm_shift_kernel, dim3((nb + 63) / 64, (d.N + 63) / 64), dim3(256), 0, s, d.N, nb,
                               W + (size_t)j * d.N * d.N, d.v, M64, Y64);
            GW_LAUNCHED("zgemm_shift_kernel");
          }
          const int rpc = (d.N + CD_CHUNKS64 - 1) / CD_CHUNKS64;
          hipLaunchKernelGGL(coldot_f64_kernel, dim3((nb + 31) / 32, CD_CHUNKS64), dim3(256), 0, s, d.N, nb, M64, Y64,
                             rpc, part);
          GW_LAUNCHED("coldot_f64_kernel");
          hipLaunchKernelGGL(coldot_sum_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, nb, CD_CHUNKS64, part,
                             q + (size_t)j * nb);
          GW_LAUNCHED("coldot_sum_kernel");
        }
        hipLaunchKernelGGL(sigma_contract_kernel, dim3(d.n_out), dim3(256), 0, s, nb, d.n_mesh, d.n_out,
                           wts + (size_t)s2 * nw, q, (long)nb, sig + (size_t)si * d.n_out);
        GW_LAUNCHED("sigma_contract_kernel");
      }
    }
    return GW_OK;
  }
  // split BF16: batches of states share each transfer's W^c words and GEMMs
  const float2* psi = static_cast<const float2*>(d.psi);
  std::vector<const float2*> pst(need.batch), pal(need.batch);
  for (int b0 = 0; b0 < d.n_states; b0 += need.batch) {
    const int g = std::min(need.batch, d.n_states - b0);
    const long ldq = tiled_sigma_cols(nb, g);
    const long col = ldq / g;
    for (int t = 0; t < d.n_k; ++t) {
      const double2* W = static_cast<const double2*>(d.W_host[t]);
      for (int i = 0; i < g; ++i) {
        const int s0 = d.state_set_host[b0 + i], n0 = d.state_band_host[b0 + i];
        pst[i] = psi + ((size_t)s0 * nb + n0) * d.R;
        pal[i] = psi + (size_t)((s0 + t) % d.n_k) * nb * d.R;
      }
      if ((st = tiled_sigma_quadforms(s, d.N, d.R, nb, g, d.n_mesh, static_cast<const float2*>(d.U), !u_tiled,
                                      pst.data(), pal.data(), W, d.v, q, quad_ws)) != GW_OK)
        return st;
      u_tiled = true;
      for (int i = 0; i < g; ++i) {
        const int s2 = (d.state_set_host[b0 + i] + t) % d.n_k;
        hipLaunchKernelGGL(sigma_contract_kernel, dim3(d.n_out), dim3(256), 0, s, nb, d.n_mesh, d.n_out,
                           wts + (size_t)s2 * nw, q + i * col, ldq, sig + (size_t)(b0 + i) * d.n_out);
        GW_LAUNCHED("sigma_contract_kernel");
      }
    }
  }
  return GW_OK;
}
