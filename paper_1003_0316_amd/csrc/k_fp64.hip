// FP64 path: transition weights, fused product + projection, weighted Hermitian
// accumulation, Hermitian mirror.  Plain FP64 FMA with LDS tiling (on gfx950
// the FP64 vector rate equals the FP64 matrix-core rate).
#include <algorithm>

#include "gw_internal.hpp"

namespace gw {
namespace {

constexpr int TM = 64;   // output tile rows
constexpr int TN = 64;   // output tile cols
constexpr int TK = 16;   // k-step
constexpr int NT = 256;  // threads per block (16 x 16, 4 x 4 outputs each)

__global__ void fill_zero_kernel(double* __restrict__ p, size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

// w[j][t] = pair_weight: 4 D / (D^2 + w_j^2), D = eps_k[n] - eps_kq[n_occ + u],
// the imaginary-axis bracket of Eq. polar_MB summed over two spins (or the
// node share of the spectral route).
__global__ void weights_f64_kernel(const double* __restrict__ eps, int n_bands, int n_occ, Chunk c,
                                   OmegaList om, double* __restrict__ w) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int T = c.T;
  if (t >= T) return;
  long g = c.tb + t;
  int n = c.n0 + (int)(g / c.nu);
  int u = c.u0 + (int)(g % c.nu);
  double d = eps[(size_t)c.k * n_bands + n] - eps[(size_t)c.kq * n_bands + n_occ + u];
  for (int j = 0; j < om.n; ++j) w[(size_t)j * T + t] = pair_weight(d, om, j);
}

// M[I][t] = sum_r U[I][r] conj(po[n][r]) pu[u][r],  t = n*nu + u  (Eq. proj_MB).
// The product conj(po) * pu is formed while staging the B tile; it is never stored.
__global__ __launch_bounds__(NT) void project_f64_kernel(int N, int R, const double2* __restrict__ U,
                                                         const double2* __restrict__ po,
                                                         const double2* __restrict__ pu, int nu, long tb, int T,
                                                         double2* __restrict__ M, long ldm) {
  __shared__ double2 As[TK][TM + 1];
  __shared__ double2 Bs[TK][TN + 1];
  const int t0 = blockIdx.x * TN;
  const int i0 = blockIdx.y * TM;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);

  for (int r0 = 0; r0 < R; r0 += TK) {
#pragma unroll
    for (int q = 0; q < (TM * TK) / NT; ++q) {
      int e = tid + q * NT;
      int kk = e % TK, ii = e / TK;
      int gi = i0 + ii, gr = r0 + kk;
      double2 val = make_double2(0.0, 0.0);
      if (gi < N && gr < R) val = U[(size_t)gi * R + gr];
      As[kk][ii] = val;
    }
#pragma unroll
    for (int q = 0; q < (TN * TK) / NT; ++q) {
      int e = tid + q * NT;
      int kk = e % TK, tt = e / TK;
      int gt = t0 + tt, gr = r0 + kk;
      double2 val = make_double2(0.0, 0.0);
      if (gt < T && gr < R) {
        long g = tb + gt;
        double2 a = po[(size_t)(g / nu) * R + gr];
        double2 b = pu[(size_t)(g % nu) * R + gr];
        // conj(a) * b
        val = make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
      }
      Bs[kk][tt] = val;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double2 av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b].x = fma(av[a].x, bv[b].x, fma(-av[a].y, bv[b].y, acc[a][b].x));
          acc[a][b].y = fma(av[a].x, bv[b].y, fma(av[a].y, bv[b].x, acc[a][b].y));
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int gi = i0 + ty + 16 * a;
    if (gi >= N) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int gt = t0 + tx + 16 * b;
      if (gt < T) M[(size_t)gi * ldm + gt] = acc[a][b];
    }
  }
}

__device__ inline void lower_tile_coords(int l, int& bi, int& bj) {
  int b = (int)((sqrt(8.0 * (double)l + 1.0) - 1.0) * 0.5);
  while ((b + 1) * (b + 2) / 2 <= l) ++b;
  while (b * (b + 1) / 2 > l) --b;
  bi = b;
  bj = l - b * (b + 1) / 2;
}

// P_j[I][J] += sum_t w[j][t] M[I][t] conj(M[J][t]) over tiles with I-block >= J-block
// (Eq. polar_MB for one chunk of transition pairs, one frequency per grid z).
__global__ __launch_bounds__(NT) void herk_f64_kernel(int N, int T, const double2* __restrict__ M, long ldm,
                                                      const double* __restrict__ w,
                                                      double2* __restrict__ P) {
  __shared__ double2 As[TK][TM + 1];
  __shared__ double2 Bs[TK][TN + 1];
  int bi, bj;
  lower_tile_coords(blockIdx.x, bi, bj);
  const int j = blockIdx.y;
  const double* wj = w + (size_t)j * T;
  const int i0 = bi * TM, c0 = bj * TN;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);

  for (int t0 = 0; t0 < T; t0 += TK) {
#pragma unroll
    for (int q = 0; q < (TM * TK) / NT; ++q) {
      int e = tid + q * NT;
      int kk = e % TK, ii = e / TK;
      int gt = t0 + kk;
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
      if (gt < T) {
        double wt = wj[gt];
        if (i0 + ii < N) {
          a = M[(size_t)(i0 + ii) * ldm + gt];
          a.x *= wt;
          a.y *= wt;
        }
        if (c0 + ii < N) b = M[(size_t)(c0 + ii) * ldm + gt];
      }
      As[kk][ii] = a;
      Bs[kk][ii] = b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double2 av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          // a * conj(b)
          acc[a][b].x = fma(av[a].x, bv[b].x, fma(av[a].y, bv[b].y, acc[a][b].x));
          acc[a][b].y = fma(av[a].y, bv[b].x, fma(-av[a].x, bv[b].y, acc[a][b].y));
        }
    }
    __syncthreads();
  }
  double2* Pj = P + (size_t)j * N * N;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int gi = i0 + ty + 16 * a;
    if (gi >= N) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int gc = c0 + tx + 16 * b;
      if (gc < N) {
        double2 p = Pj[(size_t)gi * N + gc];
        p.x += acc[a][b].x;
        p.y += acc[a][b].y;
        Pj[(size_t)gi * N + gc] = p;
      }
    }
  }
}

// Upper triangle from the lower one; real diagonal.  One 32x32 block of the
// strict lower triangle (and its transposed partner) per workgroup.
__global__ void mirror_kernel(int N, double2* __restrict__ P) {
  __shared__ double2 tile[32][33];
  int bi, bj;
  lower_tile_coords(blockIdx.x, bi, bj);
  double2* Pj = P + (size_t)blockIdx.y * N * N;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8 threads
  for (int y = ty; y < 32; y += 8) {
    int gi = bi * 32 + y, gc = bj * 32 + tx;
    if (gi < N && gc < N) tile[y][tx] = Pj[(size_t)gi * N + gc];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    // write element (bj*32 + y, bi*32 + tx) = conj(lower (bi*32+tx, bj*32+y))
    int gr = bj * 32 + y, gc = bi * 32 + tx;
    if (gr >= N || gc >= N) continue;
    if (gr < gc) {
      double2 v = tile[tx][y];
      Pj[(size_t)gr * N + gc] = make_double2(v.x, -v.y);
    } else if (gr == gc) {
      double2 v = tile[tx][y];
      Pj[(size_t)gr * N + gc] = make_double2(v.x, 0.0);
    }
  }
}

}  // namespace

int launch_fill_zero(hipStream_t s, double* p, size_t n) {
  if (n == 0) return GW_OK;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  GW_LAUNCHED("fill_zero_kernel");
  return GW_OK;
}

int launch_weights_f64(hipStream_t s, const double* eps, int n_bands, int n_occ, const Chunk& c,
                       const OmegaList& om, double* w) {
  int T = c.T;
  hipLaunchKernelGGL(weights_f64_kernel, dim3((T + 255) / 256), dim3(256), 0, s, eps, n_bands, n_occ, c,
                     om, w);
  GW_LAUNCHED("weights_f64_kernel");
  return GW_OK;
}

int launch_project_f64(hipStream_t s, int N, int R, const double2* U, const double2* po,
                       const double2* pu, int nu, long tb, int T, double2* M, long ldm) {
  dim3 grid((T + TN - 1) / TN, (N + TM - 1) / TM);
  ProfScope prof(s, "project_f64_kernel");
  hipLaunchKernelGGL(project_f64_kernel, grid, dim3(NT), 0, s, N, R, U, po, pu, nu, tb, T, M, ldm);
  GW_LAUNCHED("project_f64_kernel");
  return GW_OK;
}

int launch_herk_f64(hipStream_t s, int N, int T, const double2* M, long ldm, const double* w, int n_omega,
                    double2* P) {
  int nb = (N + TM - 1) / TM;
  dim3 grid(nb * (nb + 1) / 2, n_omega);
  ProfScope prof(s, "herk_f64_kernel");
  hipLaunchKernelGGL(herk_f64_kernel, grid, dim3(NT), 0, s, N, T, M, ldm, w, P);
  GW_LAUNCHED("herk_f64_kernel");
  return GW_OK;
}

int launch_hermitian_mirror(hipStream_t s, int N, int n_omega, double2* P) {
  int nb = (N + 31) / 32;
  dim3 grid(nb * (nb + 1) / 2, n_omega);
  hipLaunchKernelGGL(mirror_kernel, grid, dim3(256), 0, s, N, P);
  GW_LAUNCHED("mirror_kernel");
  return GW_OK;
}


// ---- finite checks ------------------------------------------------------------
namespace {
__global__ void flag_clear_kernel(unsigned* __restrict__ flag) {
  if (threadIdx.x == 0) flag[0] = 0u;
}

// flag |= 1 if any of the n values (IEEE float, or double when f64) has an
// all-ones exponent (Inf or NaN).  For doubles only the high word is read.
__global__ __launch_bounds__(256) void nonfinite_kernel(const uint32_t* __restrict__ w, size_t n, int f64,
                                                        unsigned* __restrict__ flag) {
  unsigned bad = 0u;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    if (f64) {
      const uint32_t hi = w[2 * i + 1];
      bad |= (hi & 0x7ff00000u) == 0x7ff00000u;
    } else {
      bad |= (w[i] & 0x7f800000u) == 0x7f800000u;
    }
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}
}  // namespace

int launch_flag_clear(hipStream_t s, unsigned* flag) {
  hipLaunchKernelGGL(flag_clear_kernel, dim3(1), dim3(64), 0, s, flag);
  GW_LAUNCHED("flag_clear_kernel");
  return GW_OK;
}

int launch_nonfinite(hipStream_t s, const void* p, size_t n_values, bool f64, unsigned* flag) {
  if (n_values == 0) return GW_OK;
  const unsigned blocks = (unsigned)std::min<size_t>((n_values + 255) / 256, 8192);
  hipLaunchKernelGGL(nonfinite_kernel, dim3(blocks), dim3(256), 0, s, static_cast<const uint32_t*>(p), n_values,
                     f64 ? 1 : 0, flag);
  GW_LAUNCHED("nonfinite_kernel");
  return GW_OK;
}

int read_flag(hipStream_t s, const unsigned* flag, unsigned* host) {
  GW_HIP(hipMemcpyAsync(host, flag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  GW_HIP(hipStreamSynchronize(s));
  return GW_OK;
}


namespace {
struct FreqList {
  int n;
  double w[kMaxOmega];
};

// Spectral route: P[j][e] (+)= sum_b c_jb S[b][e] with c_jb = 4 x_b / (x_b^2 +
// omega_j^2), the imaginary-axis Hilbert transform of a delta function of
// spectral weight at node energy x_b (S holds minus the node weights).  Block
// row blockIdx.y covers frequencies 8 y .. 8 y + 7; their coefficients sit in
// LDS; every element of S is read once per block row.
constexpr int SC_J = 8;
__global__ __launch_bounds__(256) void spectral_combine_kernel(size_t NN, OmegaList nodes, FreqList freq,
                                                               const double2* __restrict__ S,
                                                               double2* __restrict__ P, int accumulate) {
  __shared__ double c[SC_J][kMaxSlots];
  const int j0 = blockIdx.y * SC_J;
  const int nj = min(SC_J, freq.n - j0);
  for (int e = threadIdx.x; e < SC_J * nodes.n; e += blockDim.x) {
    const int jj = e / nodes.n, b = e % nodes.n;
    const double x = nodes.w[b], om = jj < nj ? freq.w[j0 + jj] : 0.0;
    c[jj][b] = 4.0 * x / (x * x + om * om);
  }
  __syncthreads();
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < NN; e += (size_t)gridDim.x * blockDim.x) {
    double2 acc[SC_J];
#pragma unroll
    for (int jj = 0; jj < SC_J; ++jj) acc[jj] = make_double2(0.0, 0.0);
    for (int b = 0; b < nodes.n; ++b) {
      const double2 v = S[(size_t)b * NN + e];
#pragma unroll
      for (int jj = 0; jj < SC_J; ++jj) {
        acc[jj].x = fma(c[jj][b], v.x, acc[jj].x);
        acc[jj].y = fma(c[jj][b], v.y, acc[jj].y);
      }
    }
    for (int jj = 0; jj < nj; ++jj) {
      double2* p = P + (size_t)(j0 + jj) * NN + e;
      if (accumulate) {
        const double2 o = *p;
        *p = make_double2(o.x + acc[jj].x, o.y + acc[jj].y);
      } else {
        *p = acc[jj];
      }
    }
  }
}
}  // namespace

int launch_spectral_combine(hipStream_t s, int N, const OmegaList& nodes, int n_omega, const double* omega_host,
                            const double2* S, double2* P, int accumulate) {
  FreqList f{};
  f.n = n_omega;
  for (int j = 0; j < n_omega; ++j) f.w[j] = omega_host[j];
  const size_t NN = (size_t)N * N;
  const unsigned gx = (unsigned)std::min<size_t>((NN + 255) / 256, 2048);
  hipLaunchKernelGGL(spectral_combine_kernel, dim3(gx, (n_omega + SC_J - 1) / SC_J), dim3(256), 0, s, NN, nodes, f,
                     S, P, accumulate);
  GW_LAUNCHED("spectral_combine_kernel");
  return GW_OK;
}

}  // namespace gw
