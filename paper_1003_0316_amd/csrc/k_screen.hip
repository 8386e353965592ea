// Screening in FP64 (Eqs. dielec_MB / screen_MB, Eq. W_Dyson):
//   eps = 1 - s P s  (s = sqrt(v), Hermitian positive definite for P <= 0)
//   W   = s eps^-1 s
// eps^-1 is formed in place by a blocked Gauss-Jordan sweep without pivoting on
// the lower triangle.  Sweeping pivot block p (D = A_pp^-1, C_i = A_ip D):
//   A_ij -= C_i A_pj      (i, j outside p)
//   A_ip  = C_i,  A_pj = D A_pj = C_j^H,  A_pp = -D
// After every block has been swept the matrix holds -eps^-1.  Each step is a
// rank-bp update of the lower triangle; every output element has one owner.
#include "gw_internal.hpp"

namespace gw {
namespace {

constexpr int PB = 32;   // pivot block
constexpr int UT = 64;   // update tile
constexpr int NT = 256;

__device__ inline void lower_tile(int l, int& bi, int& bj) {
  int b = (int)((sqrt(8.0 * (double)l + 1.0) - 1.0) * 0.5);
  while ((b + 1) * (b + 2) / 2 <= l) ++b;
  while (b * (b + 1) / 2 > l) --b;
  bi = b;
  bj = l - b * (b + 1) / 2;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// A = 1 - s P s on the lower triangle (upper triangle left untouched).
__global__ void build_eps_kernel(int N, const double2* __restrict__ P, const double* __restrict__ v,
                                 double2* __restrict__ A, int* __restrict__ info) {
  const size_t NN = (size_t)N * N;
  const size_t base = (size_t)blockIdx.y * NN;
  if (blockIdx.x == 0 && threadIdx.x == 0) info[blockIdx.y] = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < NN; e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e / N), j = (int)(e % N);
    if (j > i) continue;
    double sij = sqrt(v[i]) * sqrt(v[j]);
    double2 p = P[base + e];
    double2 a = make_double2(-sij * p.x, -sij * p.y);
    if (i == j) {
      a.x += 1.0;
      a.y = 0.0;
    }
    A[base + e] = a;
  }
}

// Invert the Hermitian pivot block in LDS by an unblocked sweep; D = A_pp^-1.
__global__ __launch_bounds__(1024) void pivot_kernel(int N, int c0, int bp, double2* __restrict__ A,
                                                     double2* __restrict__ Dbuf, int* __restrict__ info) {
  __shared__ double2 blk[PB][PB + 1];
  __shared__ int bad;
  const int om = blockIdx.x;
  if (info[om] != 0) return;
  double2* Aj = A + (size_t)om * N * N;
  const int r = threadIdx.x / PB, c = threadIdx.x % PB;
  if (threadIdx.x == 0) bad = 0;
  if (r < bp && c < bp) {
    double2 x;
    if (r >= c) {
      x = Aj[(size_t)(c0 + r) * N + c0 + c];
    } else {
      double2 y = Aj[(size_t)(c0 + c) * N + c0 + r];
      x = make_double2(y.x, -y.y);
    }
    if (r == c) x.y = 0.0;
    blk[r][c] = x;
  }
  __syncthreads();
  for (int k = 0; k < bp; ++k) {
    double piv = blk[k][k].x;
    double2 a_rk = make_double2(0, 0), a_kc = make_double2(0, 0), a_rc = make_double2(0, 0);
    if (r < bp && c < bp) {
      a_rk = blk[r][k];
      a_kc = blk[k][c];
      a_rc = blk[r][c];
    }
    __syncthreads();
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (threadIdx.x == 0) bad = c0 + k + 1;
      __syncthreads();
      break;
    }
    double ip = 1.0 / piv;
    if (r < bp && c < bp) {
      double2 out;
      if (r == k && c == k) {
        out = make_double2(-ip, 0.0);
      } else if (r == k) {
        out = make_double2(a_kc.x * ip, a_kc.y * ip);
      } else if (c == k) {
        out = make_double2(a_rk.x * ip, a_rk.y * ip);
      } else {
        double2 pr = cmul(a_rk, a_kc);
        out = make_double2(a_rc.x - pr.x * ip, a_rc.y - pr.y * ip);
      }
      blk[r][c] = out;
    }
    __syncthreads();
  }
  if (bad) {
    if (threadIdx.x == 0) info[om] = bad;
    return;
  }
  // blk = -A_pp^-1
  if (r < PB && c < PB) {
    double2 d = (r < bp && c < bp) ? make_double2(-blk[r][c].x, -blk[r][c].y) : make_double2(0, 0);
    Dbuf[(size_t)om * PB * PB + r * PB + c] = d;
  }
}

// C_i = A_ip D and O_i = A_ip (old) for every row i outside the pivot block.
__global__ __launch_bounds__(NT) void panel_kernel(int N, int c0, int bp, const double2* __restrict__ A,
                                                   const double2* __restrict__ Dbuf, double2* __restrict__ Cbuf,
                                                   double2* __restrict__ Obuf, const int* __restrict__ info) {
  __shared__ double2 Ds[PB][PB + 1];
  __shared__ double2 Ar[UT][PB + 1];
  const int om = blockIdx.y;
  if (info[om] != 0) return;
  const double2* Aj = A + (size_t)om * N * N;
  const int i0 = blockIdx.x * UT;
  const int c1 = c0 + bp;
  for (int e = threadIdx.x; e < PB * PB; e += NT) Ds[e / PB][e % PB] = Dbuf[(size_t)om * PB * PB + e];
  for (int e = threadIdx.x; e < UT * PB; e += NT) {
    int ii = e % UT, kk = e / UT;
    int i = i0 + ii;
    double2 x = make_double2(0, 0);
    if (i < N && kk < bp) {
      if (i >= c1) {
        x = Aj[(size_t)i * N + c0 + kk];
      } else if (i < c0) {
        double2 y = Aj[(size_t)(c0 + kk) * N + i];
        x = make_double2(y.x, -y.y);
      }
    }
    Ar[ii][kk] = x;
  }
  __syncthreads();
  double2* Cj = Cbuf + (size_t)om * N * PB;
  double2* Oj = Obuf + (size_t)om * N * PB;
  for (int e = threadIdx.x; e < UT * PB; e += NT) {
    int ii = e / PB, jj = e % PB;
    int i = i0 + ii;
    if (i >= N) continue;
    double2 s = make_double2(0, 0);
    for (int kk = 0; kk < bp; ++kk) {
      double2 pr = cmul(Ar[ii][kk], Ds[kk][jj]);
      s.x += pr.x;
      s.y += pr.y;
    }
    Cj[(size_t)i * PB + jj] = s;
    Oj[(size_t)i * PB + jj] = Ar[ii][jj];
  }
}

// Rank-bp update of the lower triangle plus the new pivot row/column/block.
__global__ __launch_bounds__(NT) void update_kernel(int N, int c0, int bp, double2* __restrict__ A,
                                                    const double2* __restrict__ Dbuf,
                                                    const double2* __restrict__ Cbuf,
                                                    const double2* __restrict__ Obuf, const int* __restrict__ info) {
  __shared__ double2 Cs[PB][UT + 1];
  __shared__ double2 Os[PB][UT + 1];
  const int om = blockIdx.y;
  if (info[om] != 0) return;
  int bi, bj;
  lower_tile(blockIdx.x, bi, bj);
  const int i0 = bi * UT, j0 = bj * UT;
  const int c1 = c0 + bp;
  double2* Aj = A + (size_t)om * N * N;
  const double2* Cj = Cbuf + (size_t)om * N * PB;
  const double2* Oj = Obuf + (size_t)om * N * PB;
  const double2* Dj = Dbuf + (size_t)om * PB * PB;
  for (int e = threadIdx.x; e < UT * PB; e += NT) {
    int ii = e / PB, kk = e % PB;
    int i = i0 + ii, j = j0 + ii;
    Cs[kk][ii] = (i < N && kk < bp) ? Cj[(size_t)i * PB + kk] : make_double2(0, 0);
    Os[kk][ii] = (j < N && kk < bp) ? Oj[(size_t)j * PB + kk] : make_double2(0, 0);
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0, 0);
  for (int kk = 0; kk < bp; ++kk) {
    double2 cv[4], ov[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) cv[a] = Cs[kk][ty + 16 * a];
#pragma unroll
    for (int b = 0; b < 4; ++b) ov[b] = Os[kk][tx + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        // C_i * conj(O_j)
        acc[a][b].x = fma(cv[a].x, ov[b].x, fma(cv[a].y, ov[b].y, acc[a][b].x));
        acc[a][b].y = fma(cv[a].y, ov[b].x, fma(-cv[a].x, ov[b].y, acc[a][b].y));
      }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int i = i0 + ty + 16 * a;
    if (i >= N) continue;
    bool ip = (i >= c0 && i < c1);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int j = j0 + tx + 16 * b;
      if (j >= N || j > i) continue;
      bool jp = (j >= c0 && j < c1);
      size_t off = (size_t)i * N + j;
      if (!ip && !jp) {
        double2 x = Aj[off];
        x.x -= acc[a][b].x;
        x.y -= acc[a][b].y;
        Aj[off] = x;
      } else if (!ip && jp) {
        Aj[off] = Cj[(size_t)i * PB + (j - c0)];
      } else if (ip && !jp) {
        double2 y = Cj[(size_t)j * PB + (i - c0)];
        Aj[off] = make_double2(y.x, -y.y);
      } else {
        double2 d = Dj[(i - c0) * PB + (j - c0)];
        Aj[off] = make_double2(-d.x, -d.y);
      }
    }
  }
}

// W = -s A s on the lower triangle (A holds -eps^-1).
__global__ void finish_kernel(int N, const double* __restrict__ v, double2* __restrict__ A) {
  const size_t NN = (size_t)N * N;
  const size_t base = (size_t)blockIdx.y * NN;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < NN; e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e / N), j = (int)(e % N);
    if (j > i) continue;
    double sij = sqrt(v[i]) * sqrt(v[j]);
    double2 a = A[base + e];
    A[base + e] = make_double2(-sij * a.x, -sij * a.y);
  }
}

}  // namespace

size_t screen_workspace_bytes(int N, int n_omega) {
  size_t d = align_up((size_t)n_omega * PB * PB * sizeof(double2));
  size_t c = align_up((size_t)n_omega * N * PB * sizeof(double2));
  return d + 2 * c;
}

int screen_run(hipStream_t s, int N, int n_omega, const double2* P, const double* v, double2* W, int* info,
               void* ws) {
  Carver cv(ws);
  double2* Dbuf = cv.take<double2>((size_t)n_omega * PB * PB);
  double2* Cbuf = cv.take<double2>((size_t)n_omega * N * PB);
  double2* Obuf = cv.take<double2>((size_t)n_omega * N * PB);
  size_t NN = (size_t)N * N;
  unsigned eb = (unsigned)std::min<size_t>((NN + 255) / 256, 8192);
  hipLaunchKernelGGL(build_eps_kernel, dim3(eb, n_omega), dim3(256), 0, s, N, P, v, W, info);
  GW_LAUNCHED("build_eps_kernel");
  const int nb = (N + UT - 1) / UT;
  const int ntiles = nb * (nb + 1) / 2;
  for (int c0 = 0; c0 < N; c0 += PB) {
    int bp = std::min(PB, N - c0);
    hipLaunchKernelGGL(pivot_kernel, dim3(n_omega), dim3(PB * PB), 0, s, N, c0, bp, W, Dbuf, info);
    GW_LAUNCHED("pivot_kernel");
    hipLaunchKernelGGL(panel_kernel, dim3(nb, n_omega), dim3(NT), 0, s, N, c0, bp, W, Dbuf, Cbuf, Obuf, info);
    GW_LAUNCHED("panel_kernel");
    ProfScope prof(s, "update_kernel");
    hipLaunchKernelGGL(update_kernel, dim3(ntiles, n_omega), dim3(NT), 0, s, N, c0, bp, W, Dbuf, Cbuf, Obuf,
                       info);
    GW_LAUNCHED("update_kernel");
  }
  hipLaunchKernelGGL(finish_kernel, dim3(eb, n_omega), dim3(256), 0, s, N, v, W);
  GW_LAUNCHED("finish_kernel");
  return launch_hermitian_mirror(s, N, n_omega, W);
}

}  // namespace gw
