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

constexpr int PB = 64;   // pivot block
constexpr int UT = 64;   // update tile (4 waves of 32 x 32); equal to PB
static_assert(PB == UT, "the update's fast path assumes pivot blocks aligned to update tiles");
constexpr int PT = 32;   // rows per panel workgroup
constexpr int NT = 256;
constexpr int PV = 1024; // pivot threads

typedef double dbl4 __attribute__((ext_vector_type(4)));

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

// Panel layout of C and O: element (row i, pivot column k) at
// ((k / 4) * Nr + i) * 4 + k % 4 (complex), Nr = rows rounded up to UT.  The 64
// lanes of an FP64 16x16x4 MFMA fragment (row l % 16, k l / 16) then read one
// contiguous kilobyte.
__device__ inline size_t panel_idx(int Nr, int i, int k) {
  return ((size_t)(k >> 2) * Nr + i) * 4 + (k & 3);
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

// Invert the Hermitian pivot block in LDS by an unblocked sweep; D = A_pp^-1
// (stored negated, zero-padded to PB x PB).  Each thread owns PB*PB/PV
// elements.
__global__ __launch_bounds__(PV) void pivot_kernel(int N, int c0, int bp, double2* __restrict__ A,
                                                   double2* __restrict__ Dbuf, int* __restrict__ info) {
  constexpr int EPT = PB * PB / PV;
  __shared__ double2 blk[PB][PB + 1];
  __shared__ int bad;
  const int om = blockIdx.x;
  if (info[om] != 0) return;
  double2* Aj = A + (size_t)om * N * N;
  if (threadIdx.x == 0) bad = 0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + q * PV, r = e / PB, c = e % PB;
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
  }
  __syncthreads();
  for (int k = 0; k < bp; ++k) {
    const double piv = blk[k][k].x;
    double2 a_rk[EPT], a_kc[EPT], a_rc[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + q * PV, r = e / PB, c = e % PB;
      a_rk[q] = a_kc[q] = a_rc[q] = make_double2(0, 0);
      if (r < bp && c < bp) {
        a_rk[q] = blk[r][k];
        a_kc[q] = blk[k][c];
        a_rc[q] = blk[r][c];
      }
    }
    __syncthreads();
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (threadIdx.x == 0) bad = c0 + k + 1;
      __syncthreads();
      break;
    }
    const double ip = 1.0 / piv;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + q * PV, r = e / PB, c = e % PB;
      if (r < bp && c < bp) {
        double2 out;
        if (r == k && c == k) {
          out = make_double2(-ip, 0.0);
        } else if (r == k) {
          out = make_double2(a_kc[q].x * ip, a_kc[q].y * ip);
        } else if (c == k) {
          out = make_double2(a_rk[q].x * ip, a_rk[q].y * ip);
        } else {
          double2 pr = cmul(a_rk[q], a_kc[q]);
          out = make_double2(a_rc[q].x - pr.x * ip, a_rc[q].y - pr.y * ip);
        }
        blk[r][c] = out;
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (threadIdx.x == 0) info[om] = bad;
    return;
  }
  // blk = -A_pp^-1
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + q * PV, r = e / PB, c = e % PB;
    double2 d = (r < bp && c < bp) ? make_double2(-blk[r][c].x, -blk[r][c].y) : make_double2(0, 0);
    Dbuf[(size_t)om * PB * PB + r * PB + c] = d;
  }
}

// C_i = A_ip D and O_i = A_ip (old) for every row i < Nr outside the pivot
// block, in the panel layout; rows inside the block or past N and pivot
// columns past bp are zero.
__global__ __launch_bounds__(NT) void panel_kernel(int N, int Nr, int c0, int bp, const double2* __restrict__ A,
                                                   const double2* __restrict__ Dbuf, double2* __restrict__ Cbuf,
                                                   double2* __restrict__ Obuf, const int* __restrict__ info) {
  __shared__ double2 Ar[PT][PB + 1];
  const int om = blockIdx.y;
  if (info[om] != 0) return;
  const double2* Aj = A + (size_t)om * N * N;
  const double2* Dj = Dbuf + (size_t)om * PB * PB;
  const int i0 = blockIdx.x * PT;
  const int c1 = c0 + bp;
  for (int e = threadIdx.x; e < PT * PB; e += NT) {
    int ii = e % PT, kk = e / PT;
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
  double2* Cj = Cbuf + (size_t)om * Nr * PB;
  double2* Oj = Obuf + (size_t)om * Nr * PB;
  for (int e = threadIdx.x; e < PT * PB; e += NT) {
    int ii = e / PB, jj = e % PB;
    int i = i0 + ii;
    if (i >= Nr) continue;
    double2 s = make_double2(0, 0);
    for (int kk = 0; kk < bp; ++kk) {
      double2 pr = cmul(Ar[ii][kk], Dj[kk * PB + jj]);
      s.x += pr.x;
      s.y += pr.y;
    }
    Cj[panel_idx(Nr, i, jj)] = s;
    Oj[panel_idx(Nr, i, jj)] = Ar[ii][jj];
  }
}

// Rank-bp update of the lower triangle, A_ij -= sum_k C_ik conj(O_jk), on FP64
// MFMAs (16x16x4; Re = Cr Or + Ci Oi, Im = Ci Or - Cr Oi), plus the new pivot
// row/column/block.  Wave w of the 64 x 64 tile owns rows 32 (w / 2) and
// columns 32 (w % 2) onwards as 2 x 2 blocks of 16 x 16.  Fragment layout of
// the FP64 16x16x4 MFMA: A[i][k] and B[k][j] in lane (i or j) + 16 k; the
// result D[i][j] in lane j + 16 (i % 4), register i / 4.
__global__ __launch_bounds__(NT) void update_kernel(int N, int Nr, int c0, int bp, double2* __restrict__ A,
                                                    const double2* __restrict__ Dbuf,
                                                    const double2* __restrict__ Cbuf,
                                                    const double2* __restrict__ Obuf, const int* __restrict__ info) {
  const int om = blockIdx.y;
  if (info[om] != 0) return;
  int bi, bj;
  lower_tile(blockIdx.x, bi, bj);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rb = bi * UT + 32 * (w >> 1), cb = bj * UT + 32 * (w & 1);
  const int l16 = lane & 15, lk = lane >> 4;
  const int c1 = c0 + bp;
  double2* Aj = A + (size_t)om * N * N;
  const double2* Cj = Cbuf + (size_t)om * Nr * PB;
  const double2* Oj = Obuf + (size_t)om * Nr * PB;
  const double2* Dj = Dbuf + (size_t)om * PB * PB;

  dbl4 re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      re[a][b] = dbl4{0, 0, 0, 0};
      im[a][b] = dbl4{0, 0, 0, 0};
    }
  // All PB / 4 steps, unrolled (panel columns past bp are zero, so a short
  // last pivot block adds exact zeros); no loop-carried accumulators.
#pragma unroll
  for (int ks = 0; ks < PB / 4; ++ks) {
    double2 cv[2], ov[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) cv[a] = Cj[((size_t)ks * Nr + rb + 16 * a + l16) * 4 + lk];
#pragma unroll
    for (int b = 0; b < 2; ++b) ov[b] = Oj[((size_t)ks * Nr + cb + 16 * b + l16) * 4 + lk];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(cv[a].x, ov[b].x, re[a][b], 0, 0, 0);
        re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(cv[a].y, ov[b].y, re[a][b], 0, 0, 0);
        im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(cv[a].y, ov[b].x, im[a][b], 0, 0, 0);
        im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-cv[a].x, ov[b].y, im[a][b], 0, 0, 0);
      }
  }
  // The pivot block [c0, c0 + bp) lies inside tile row / column c0 / UT (c0 is a
  // multiple of PB = UT); every other tile is a plain read-modify-write, done
  // with all loads in flight before the stores.
  if (bi * UT != c0 && bj * UT != c0) {
    double2 x[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int i = rb + 16 * a + 4 * r + lk, j = cb + 16 * b + l16;
          x[a][b][r] = (i < N && j <= i) ? Aj[(size_t)i * N + j] : make_double2(0, 0);
        }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int i = rb + 16 * a + 4 * r + lk, j = cb + 16 * b + l16;
          if (i < N && j <= i)
            Aj[(size_t)i * N + j] = make_double2(x[a][b][r].x - re[a][b][r], x[a][b][r].y - im[a][b][r]);
        }
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rb + 16 * a + 4 * r + lk;
      if (i >= N) continue;
      const bool ip = (i >= c0 && i < c1);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = cb + 16 * b + l16;
        if (j >= N || j > i) continue;
        const bool jp = (j >= c0 && j < c1);
        const size_t off = (size_t)i * N + j;
        if (!ip && !jp) {
          double2 x = Aj[off];
          x.x -= re[a][b][r];
          x.y -= im[a][b][r];
          Aj[off] = x;
        } else if (!ip && jp) {
          Aj[off] = Cj[panel_idx(Nr, i, j - c0)];
        } else if (ip && !jp) {
          double2 y = Cj[panel_idx(Nr, j, i - c0)];
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
  const size_t Nr = (size_t)((N + UT - 1) / UT) * UT;
  size_t d = align_up((size_t)n_omega * PB * PB * sizeof(double2));
  size_t c = align_up((size_t)n_omega * Nr * PB * sizeof(double2));
  return d + 2 * c;
}

int screen_run(hipStream_t s, int N, int n_omega, const double2* P, const double* v, double2* W, int* info,
               void* ws) {
  const int nb = (N + UT - 1) / UT;
  const int Nr = nb * UT;
  Carver cv(ws);
  double2* Dbuf = cv.take<double2>((size_t)n_omega * PB * PB);
  double2* Cbuf = cv.take<double2>((size_t)n_omega * Nr * PB);
  double2* Obuf = cv.take<double2>((size_t)n_omega * Nr * PB);
  size_t NN = (size_t)N * N;
  unsigned eb = (unsigned)std::min<size_t>((NN + 255) / 256, 8192);
  hipLaunchKernelGGL(build_eps_kernel, dim3(eb, n_omega), dim3(256), 0, s, N, P, v, W, info);
  GW_LAUNCHED("build_eps_kernel");
  const int ntiles = nb * (nb + 1) / 2;
  const int npanel = (Nr + PT - 1) / PT;
  for (int c0 = 0; c0 < N; c0 += PB) {
    int bp = std::min(PB, N - c0);
    hipLaunchKernelGGL(pivot_kernel, dim3(n_omega), dim3(PV), 0, s, N, c0, bp, W, Dbuf, info);
    GW_LAUNCHED("pivot_kernel");
    hipLaunchKernelGGL(panel_kernel, dim3(npanel, n_omega), dim3(NT), 0, s, N, Nr, c0, bp, W, Dbuf, Cbuf, Obuf,
                       info);
    GW_LAUNCHED("panel_kernel");
    ProfScope prof(s, "update_kernel");
    hipLaunchKernelGGL(update_kernel, dim3(ntiles, n_omega), dim3(NT), 0, s, N, Nr, c0, bp, W, Dbuf, Cbuf, Obuf,
                       info);
    GW_LAUNCHED("update_kernel");
  }
  hipLaunchKernelGGL(finish_kernel, dim3(eb, n_omega), dim3(256), 0, s, N, v, W);
  GW_LAUNCHED("finish_kernel");
  return launch_hermitian_mirror(s, N, n_omega, W);
}

}  // namespace gw
