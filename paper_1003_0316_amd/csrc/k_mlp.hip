// Small perceptron for the high-band surrogate: forward, backward, loss and
// Adam on the gfx950 matrix cores.
//
// Network: h1 = silu(x W1 + b1), h2 = silu(h1 W2 + b2), y = h2 W3 + b3,
// silu(z) = z * sigmoid(z).  FP32 master parameters; the matrix products use
// BF16 copies of the weights.  Activations and gradients stay FP32: a product
// of an FP32 operand with a BF16 weight is formed as hi*w + lo*w with
// hi = bf16(a), lo = bf16(a - hi), so only the weights are rounded.  Weight
// gradients (activation^T x gradient) run on FP32 MFMA.  Every output has one
// owner and reductions run in a fixed order (deterministic).
#include <algorithm>

#include "gw_internal.hpp"

namespace gw {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigm(z); }
__device__ inline float dsilu(float z) {
  float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

enum Epi { EPI_HIDDEN = 0, EPI_OUTPUT = 1, EPI_BWD_HIDDEN = 2, EPI_BWD_INPUT = 3 };

// out[r][c] = sum_k A[r][k] B[c][k] for c < nout, k < K (multiples of 32,
// nout <= 256); A FP32 (row stride lda), B BF16 [nout][K].  Each wave owns 16
// rows x nout columns; a workgroup of 4 waves 64 rows.
template <int NOUT>
__global__ __launch_bounds__(256) void rowgemm_kernel(int rows, int K, const float* __restrict__ A, int lda,
                                                      const uint16_t* __restrict__ B, const float* __restrict__ bias,
                                                      int epi, const float* __restrict__ Zin, float* __restrict__ out0,
                                                      float* __restrict__ out1) {
  constexpr int NT = NOUT / 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r0 = blockIdx.x * 64 + wv * 16;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  floatx4 acc[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int arow = r0 + lr;
  const bool rok = arow < rows;
  for (int s = 0; s < K; s += 32) {
    float a[8];
    if (rok) {
      const float4* p = reinterpret_cast<const float4*>(A + (size_t)arow * lda + s + lk);
      float4 x0 = p[0], x1 = p[1];
      a[0] = x0.x; a[1] = x0.y; a[2] = x0.z; a[3] = x0.w;
      a[4] = x1.x; a[5] = x1.y; a[6] = x1.z; a[7] = x1.w;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = 0.f;
    }
    bf16x8 ah, al;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 h = (__bf16)a[e];
      ah[e] = h;
      al[e] = (__bf16)(a[e] - (float)h);
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      uint4 bw = *reinterpret_cast<const uint4*>(B + (size_t)(c * 16 + lr) * K + s + lk);
      bf16x8 b = __builtin_bit_cast(bf16x8, bw);
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b, acc[c], 0, 0, 0);
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, acc[c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    const int col = c * 16 + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + (lane >> 4) * 4 + v;
      if (row >= rows) continue;
      const size_t o = (size_t)row * NOUT + col;
      float x = acc[c][v];
      if (epi == EPI_HIDDEN) {
        float z = x + bias[col];
        out0[o] = z;
        out1[o] = silu(z);
      } else if (epi == EPI_OUTPUT) {
        out0[o] = x + bias[col];
      } else if (epi == EPI_BWD_HIDDEN) {
        out0[o] = x * dsilu(Zin[o]);
      } else {
        out0[o] = x;
      }
    }
  }
}

// dW[k][j] = sum_r A[r][k] G[r][j]  (A [rows][K], G [rows][n]; 32x32 tile per
// workgroup, the 4 waves take interleaved row pairs, partial tiles are summed in
// LDS in a fixed order).
__global__ __launch_bounds__(256) void wgrad_kernel(int rows, int K, int n, const float* __restrict__ A,
                                                    const float* __restrict__ G, float* __restrict__ dW) {
  __shared__ float part[4][32][33];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int i = lane & 31, kk = lane >> 5;
  floatx16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int p = wv; 2 * p < rows; p += 4) {
    int r = 2 * p + kk;
    float a = r < rows ? A[(size_t)r * K + k0 + i] : 0.f;
    float g = r < rows ? G[(size_t)r * n + j0 + i] : 0.f;
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, g, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    part[wv][row][lane & 31] = acc[v];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 1024; e += 256) {
    int row = e >> 5, col = e & 31;
    float s = ((part[0][row][col] + part[1][row][col]) + part[2][row][col]) + part[3][row][col];
    dW[(size_t)(k0 + row) * n + j0 + col] = s;
  }
}

// db[j] = sum_r G[r][j], fixed order.
__global__ void colsum_kernel(int rows, int n, const float* __restrict__ G, float* __restrict__ db) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += G[(size_t)r * n + j];
  db[j] = s;
}

// L = (1/rows) sum 0.5 m (y-t)^2 over the first n_used of n columns; dY = m (y-t) / rows.
__global__ __launch_bounds__(1024) void loss_kernel(int rows, int n, int n_used, const float* __restrict__ Y,
                                                    const float* __restrict__ T, const float* __restrict__ mask,
                                                    float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float red[1024];
  const float inv = 1.0f / (float)rows;
  float s = 0.f;
  const size_t total = (size_t)rows * n;
  for (size_t e = threadIdx.x; e < total; e += 1024) {
    int c = (int)(e % n);
    size_t r = e / n;
    float g = 0.f;
    if (c < n_used) {
      float m = mask ? mask[r * n_used + c] : 1.0f;
      float d = Y[e] - T[r * n_used + c];
      g = m * d * inv;
      s += 0.5f * m * d * d;
    }
    dY[e] = g;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv;
}

struct MlpDims {
  int n_in, width, n_out;
  size_t off_w1, off_b1, off_w2, off_b2, off_w3, off_b3, n_params;
  size_t bo_w1, bo_w2, bo_w3, n_bf16;
};

MlpDims dims_of(int n_in, int width, int n_out) {
  MlpDims d;
  d.n_in = n_in;
  d.width = width;
  d.n_out = n_out;
  d.off_w1 = 0;
  d.off_b1 = d.off_w1 + (size_t)n_in * width;
  d.off_w2 = d.off_b1 + width;
  d.off_b2 = d.off_w2 + (size_t)width * width;
  d.off_w3 = d.off_b2 + width;
  d.off_b3 = d.off_w3 + (size_t)width * n_out;
  d.n_params = d.off_b3 + n_out;
  d.bo_w1 = 0;
  d.bo_w2 = (size_t)n_in * width;
  d.bo_w3 = d.bo_w2 + (size_t)width * width;
  d.n_bf16 = d.bo_w3 + (size_t)width * n_out;
  return d;
}

__device__ inline uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

// BF16 copies of one weight matrix W [K][n]: wk (same layout) and wt ([n][K]).
__device__ inline void store_copies(const MlpDims& d, size_t e, float p, uint16_t* wt, uint16_t* wk) {
  size_t off, bo;
  int K, n;
  if (e >= d.off_w1 && e < d.off_b1) { off = d.off_w1; bo = d.bo_w1; K = d.n_in; n = d.width; }
  else if (e >= d.off_w2 && e < d.off_b2) { off = d.off_w2; bo = d.bo_w2; K = d.width; n = d.width; }
  else if (e >= d.off_w3 && e < d.off_b3) { off = d.off_w3; bo = d.bo_w3; K = d.width; n = d.n_out; }
  else return;
  size_t q = e - off;
  int k = (int)(q / n), j = (int)(q % n);
  uint16_t b = bf16_bits(p);
  wk[bo + q] = b;
  wt[bo + (size_t)j * K + k] = b;
}

__global__ void adam_kernel(MlpDims d, float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2,
                            uint16_t* __restrict__ wt, uint16_t* __restrict__ wk) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < d.n_params; e += (size_t)gridDim.x * blockDim.x) {
    float ge = g[e];
    float me = b1 * m[e] + (1.f - b1) * ge;
    float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    float pe = p[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    p[e] = pe;
    store_copies(d, e, pe, wt, wk);
  }
}

__global__ void sync_bf16_kernel(MlpDims d, const float* __restrict__ p, uint16_t* __restrict__ wt,
                                 uint16_t* __restrict__ wk) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < d.n_params; e += (size_t)gridDim.x * blockDim.x)
    store_copies(d, e, p[e], wt, wk);
}

int launch_rowgemm(hipStream_t s, int nout, int rows, int K, const float* A, int lda, const uint16_t* B,
                   const float* bias, int epi, const float* Zin, float* out0, float* out1) {
  dim3 grid((rows + 63) / 64);
  switch (nout) {
#define GW_ROWGEMM_CASE(NO)                                                                                     \
  case NO:                                                                                                      \
    hipLaunchKernelGGL(rowgemm_kernel<NO>, grid, dim3(256), 0, s, rows, K, A, lda, B, bias, epi, Zin, out0,    \
                       out1);                                                                                   \
    break;
    GW_ROWGEMM_CASE(32)
    GW_ROWGEMM_CASE(64)
    GW_ROWGEMM_CASE(128)
    GW_ROWGEMM_CASE(256)
#undef GW_ROWGEMM_CASE
    default:
      return fail(GW_ERR_UNSUPPORTED, "mlp: layer width must be 32, 64, 128 or 256");
  }
  GW_LAUNCHED("rowgemm_kernel");
  return GW_OK;
}

int launch_wgrad(hipStream_t s, int rows, int K, int n, const float* A, const float* G, float* dW, float* db) {
  hipLaunchKernelGGL(wgrad_kernel, dim3(K / 32, n / 32), dim3(256), 0, s, rows, K, n, A, G, dW);
  GW_LAUNCHED("wgrad_kernel");
  hipLaunchKernelGGL(colsum_kernel, dim3((n + 255) / 256), dim3(256), 0, s, rows, n, G, db);
  GW_LAUNCHED("colsum_kernel");
  return GW_OK;
}

bool valid_dims(int n_in, int width, int n_out) {
  auto ok = [](int x) { return x == 32 || x == 64 || x == 128 || x == 256; };
  return ok(n_in) && ok(width) && ok(n_out);
}

int check_mlp(const gw_mlp* m, bool need_adam) {
  if (!m) return fail(GW_ERR_INVALID_ARG, "mlp: descriptor is NULL");
  if (!valid_dims(m->n_in, m->width, m->n_out))
    return fail(GW_ERR_INVALID_ARG, "mlp: n_in, width, n_out must each be 32, 64, 128 or 256");
  if (!m->master || !m->wt || !m->wk) return fail(GW_ERR_INVALID_ARG, "mlp: null parameter pointer");
  if (need_adam && (!m->adam_m || !m->adam_v)) return fail(GW_ERR_INVALID_ARG, "mlp: null Adam moment pointer");
  return GW_OK;
}

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" {

int gw_mlp_sizes(int n_in, int width, int n_out, size_t* n_params, size_t* n_bf16) {
  if (!n_params || !n_bf16) return fail(GW_ERR_INVALID_ARG, "gw_mlp_sizes: null output");
  if (!valid_dims(n_in, width, n_out))
    return fail(GW_ERR_INVALID_ARG, "gw_mlp_sizes: n_in, width, n_out must each be 32, 64, 128 or 256");
  MlpDims d = dims_of(n_in, width, n_out);
  *n_params = d.n_params;
  *n_bf16 = d.n_bf16;
  return GW_OK;
}

int gw_mlp_sync_bf16(void* stream, const gw_mlp* m) {
  int st = check_mlp(m, false);
  if (st != GW_OK) return st;
  MlpDims d = dims_of(m->n_in, m->width, m->n_out);
  hipLaunchKernelGGL(sync_bf16_kernel, dim3((unsigned)std::min<size_t>((d.n_params + 255) / 256, 4096)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), d, m->master, m->wt, m->wk);
  GW_LAUNCHED("sync_bf16_kernel");
  return GW_OK;
}

int gw_mlp_forward(void* stream, const gw_mlp* m, const float* X, int rows, float* Y, float* act) {
  int st = check_mlp(m, false);
  if (st != GW_OK) return st;
  if (rows < 1 || !X || !Y || !act) return fail(GW_ERR_INVALID_ARG, "gw_mlp_forward: rows >= 1, X, Y, act required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MlpDims d = dims_of(m->n_in, m->width, m->n_out);
  const size_t rw = (size_t)rows * d.width;
  float *Z1 = act, *H1 = act + rw, *Z2 = act + 2 * rw, *H2 = act + 3 * rw;
  if ((st = launch_rowgemm(s, d.width, rows, d.n_in, X, d.n_in, m->wt + d.bo_w1, m->master + d.off_b1, EPI_HIDDEN,
                           nullptr, Z1, H1)) != GW_OK)
    return st;
  if ((st = launch_rowgemm(s, d.width, rows, d.width, H1, d.width, m->wt + d.bo_w2, m->master + d.off_b2, EPI_HIDDEN,
                           nullptr, Z2, H2)) != GW_OK)
    return st;
  return launch_rowgemm(s, d.n_out, rows, d.width, H2, d.width, m->wt + d.bo_w3, m->master + d.off_b3, EPI_OUTPUT,
                        nullptr, Y, nullptr);
}

int gw_mlp_loss(void* stream, int rows, int n_out, int n_used, const float* Y, const float* T, const float* mask,
                float* dY, float* loss) {
  if (rows < 1 || n_out < 1 || n_used < 1 || n_used > n_out || !Y || !T || !dY || !loss)
    return fail(GW_ERR_INVALID_ARG, "gw_mlp_loss: bad sizes or null pointer");
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), rows, n_out, n_used, Y, T,
                     mask, dY, loss);
  GW_LAUNCHED("loss_kernel");
  return GW_OK;
}

int gw_mlp_workspace_size(int rows, int width, size_t* bytes) {
  if (!bytes || rows < 1 || width < 1) return fail(GW_ERR_INVALID_ARG, "gw_mlp_workspace_size: bad arguments");
  *bytes = 2 * align_up((size_t)rows * width * sizeof(float));
  return GW_OK;
}

int gw_mlp_backward(void* stream, const gw_mlp* m, const float* X, const float* act, const float* dY, int rows,
                    float* grad, float* dX, void* ws, size_t ws_bytes) {
  int st = check_mlp(m, false);
  if (st != GW_OK) return st;
  if (rows < 1 || !X || !act || !dY || !grad) return fail(GW_ERR_INVALID_ARG, "gw_mlp_backward: bad arguments");
  size_t need = 0;
  gw_mlp_workspace_size(rows, m->width, &need);
  if (!ws || ws_bytes < need) return fail(GW_ERR_WORKSPACE, "gw_mlp_backward: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MlpDims d = dims_of(m->n_in, m->width, m->n_out);
  const size_t rw = (size_t)rows * d.width;
  const float *Z1 = act, *H1 = act + rw, *Z2 = act + 2 * rw, *H2 = act + 3 * rw;
  Carver cv(ws);
  float* dZ2 = cv.take<float>(rw);
  float* dZ1 = cv.take<float>(rw);
  if ((st = launch_wgrad(s, rows, d.width, d.n_out, H2, dY, grad + d.off_w3, grad + d.off_b3)) != GW_OK) return st;
  if ((st = launch_rowgemm(s, d.width, rows, d.n_out, dY, d.n_out, m->wk + d.bo_w3, nullptr, EPI_BWD_HIDDEN, Z2, dZ2,
                           nullptr)) != GW_OK)
    return st;
  if ((st = launch_wgrad(s, rows, d.width, d.width, H1, dZ2, grad + d.off_w2, grad + d.off_b2)) != GW_OK) return st;
  if ((st = launch_rowgemm(s, d.width, rows, d.width, dZ2, d.width, m->wk + d.bo_w2, nullptr, EPI_BWD_HIDDEN, Z1, dZ1,
                           nullptr)) != GW_OK)
    return st;
  if ((st = launch_wgrad(s, rows, d.n_in, d.width, X, dZ1, grad + d.off_w1, grad + d.off_b1)) != GW_OK) return st;
  if (dX)
    return launch_rowgemm(s, d.n_in, rows, d.width, dZ1, d.width, m->wk + d.bo_w1, nullptr, EPI_BWD_INPUT, nullptr, dX,
                          nullptr);
  return GW_OK;
}

int gw_mlp_adam_step(void* stream, const gw_mlp* m, const float* grad, float lr, float b1, float b2, float eps,
                     int step) {
  int st = check_mlp(m, true);
  if (st != GW_OK) return st;
  if (!grad || step < 1 || !(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return fail(GW_ERR_INVALID_ARG, "gw_mlp_adam_step: bad hyper-parameters");
  MlpDims d = dims_of(m->n_in, m->width, m->n_out);
  float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)std::min<size_t>((d.n_params + 255) / 256, 4096)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), d, m->master, m->adam_m, m->adam_v, grad, lr, b1, b2, eps, c1,
                     c2, m->wt, m->wk);
  GW_LAUNCHED("adam_kernel");
  return GW_OK;
}

}  // extern "C"
