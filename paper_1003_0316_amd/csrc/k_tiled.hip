// Split-BF16 path on pre-tiled operands.
//
// The two contractions of the method,
//   projection    (Eq. proj_MB)   M[I][t]   = sum_r U[I][r] F_t(r),
//                                 F_t(r)    = conj(psi_n(r)) psi_n'(r),
//   accumulation  (Eq. polar_MB)  P_j[I][J] += sum_t w_j(t) M[I][t] conj(M[J][t]),
// run on one GEMM core whose operands are prepared by streaming kernels in
// the exact layout the core copies into LDS: bf16 hi/lo words (x = hi + lo),
// complex values interleaved (re in the low half of a dword, im in the high
// half), and every complex sign/permutation pattern the MFMA embedding needs
// already applied.  The core then only moves contiguous 16-byte vectors and
// issues MFMAs.
//
// Complex products as real MFMAs: with the reduction index carrying (re, im)
// pairs, sum_k a_k b_k over interleaved rows gives
//   [re(a), -im(a)] . [re(b), im(b)] = Re(a b)          (A word: conj a)
//   [im(a),  re(a)] . [re(b), im(b)] = Im(a b)          (A word: swap a)
// and for the accumulation, with X = s M and s_j(t) = sqrt(-w_j(t)) (the
// weights are negative for every occupied-unoccupied pair of an insulator),
// P_j -= X X^H:
//   [re x_I, im x_I] . [re x_J, im x_J]   = Re(x_I conj x_J)   (A word: x)
//   [im x_I, -re x_I] . [re x_J, im x_J]  = Im(x_I conj x_J)   (A word: -i x)
// Each real product is split as hi*hi + hi*lo + lo*hi with FP32 accumulation.
//
// Tiled operand layout ("block-stage" = 128 rows x 16 complex k):
//   dword index inside one word of a block-stage:
//     ((s * 2 + h) * 128 + row) * 4 + j,   k = 8 s + 4 h + j
//   i.e. the 32x32x16 MFMA fragment of lane (row = l % 32, h = l / 32) for
//   step s is one aligned 16-byte vector, and 32 consecutive rows are 512
//   contiguous bytes (LDS reads without bank conflicts).
//   A-side arrays hold 4 words per block-stage (conj|swap or x|-ix, each
//   hi then lo); B-side arrays hold hi, lo (the product array) or the same
//   4-word array with only its first two words read.
#include "gw_mfma.hpp"

#include <algorithm>
#include <type_traits>

namespace gw {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TR = 128;               // rows per operand block
constexpr int TK = 16;                // complex k per stage
constexpr int WD = TR * TK;           // dwords per word per block-stage (2048 = 8 KB)
constexpr int GT = 256;               // GEMM workgroup: 4 waves, 2 (rows) x 2 (cols)
constexpr int TM = 128, TN = 256;     // GEMM output tile (rows from A, cols from B)
constexpr int LDS_STAGE = 8 * WD;     // dwords per LDS stage: A 4 words + B 2 halves x 2 words
constexpr size_t kGemmLds = 2 * LDS_STAGE * sizeof(uint32_t);   // double-buffered, 128 KB

__device__ inline uint32_t pack_bf16(float a, float b) {
  bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
// x = hi + lo with hi = bf16(x) (round to nearest even) and lo = bf16(x - hi).
__device__ inline void split2(float x, float& h, float& l) {
  h = (float)(__bf16)x;
  l = x - h;
}
__device__ inline int lane_off(int sh, int row) { return (sh * TR + row) * 4; }

// Three-multiplication form of the complex products (Gauss): with real planes
// a = re, b = im of one operand and c, d of the other,
//   T1 = sum a c,  T2 = sum b d,  T3 = sum (a + b)(c + d)   (projection)
//   Re = T1 - T2,  Im = T3 - T1 - T2,
// and for the accumulation's x conj(y) the second operand enters as (c, d,
// c - d), giving Re = T1 + T2, Im = T3 - T1 + T2: three real products per
// complex product instead of four.  Operands are real planes, one "plane word"
// per block-stage holds 128 rows x 16 real values (4 KB): dword
// (h * 128 + row) * 4 + j packs k = 8 h + 2 j and 8 h + 2 j + 1 (low, high
// half), so the 32x32x16 MFMA fragment of lane (row = l % 32, h = l / 32) is
// one aligned 16-byte vector.  Every plane is split hi + lo as above.
constexpr int HWD = TR * 8;           // dwords per plane word per block-stage (1024 = 4 KB)
__device__ inline int lane_off3(int h, int row) { return (h * TR + row) * 4; }

// Plane words in BF16 (W = 0) or FP16 (W = 1).  FP16 words carry a power of
// two scale per operand row (or pair) that puts the row's largest value in
// [2^13, 2^14), so hi stays far below FP16's maximum and lo in its normal
// range, and both splits accumulate into one FP32 set; the epilogues divide
// the scales out.
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

__device__ inline uint32_t pack_f16(float a, float b) {
  halfx2 v = {(_Float16)a, (_Float16)b};
  return __builtin_bit_cast(uint32_t, v);
}

template <int W>
__device__ inline uint32_t pack_w(float a, float b) {
  if constexpr (W == 0) return pack_bf16(a, b);
  else return pack_f16(a, b);
}

template <int W>
__device__ inline void split_w(float x, float& h, float& l) {
  if constexpr (W == 0) h = (float)(__bf16)x;
  else h = (float)(_Float16)x;
  l = x - h;
}

// power of two s with mx * s in [2^13, 2^14) (1 if mx is 0 or not finite)
__device__ inline float pow2_scale14(float mx) {
  if (!(mx > 0.f) || !isfinite(mx)) return 1.f;
  int e;
  frexpf(mx, &e);
  return ldexpf(1.f, 14 - e);
}

// 8 values -> hi and lo plane-word vectors.
template <int W>
__device__ inline void pack_plane(const float (&v)[8], uint4& hi, uint4& lo) {
  float h[8], l[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) split_w<W>(v[q], h[q], l[q]);
  hi = make_uint4(pack_w<W>(h[0], h[1]), pack_w<W>(h[2], h[3]), pack_w<W>(h[4], h[5]), pack_w<W>(h[6], h[7]));
  lo = make_uint4(pack_w<W>(l[0], l[1]), pack_w<W>(l[2], l[3]), pack_w<W>(l[4], l[5]), pack_w<W>(l[6], l[7]));
}

// ------------------------------------------------------------ operand tiling

// U (c64 [N][R]) -> A-side words [nI][nst][4][WD]: conj(U) hi, lo, swap(U) hi, lo.
// Rows >= N and k >= R are zero.
__global__ void tile_u_kernel(int N, int R, int nI, int nst, const float2* __restrict__ U,
                              uint32_t* __restrict__ out) {
  const size_t total = (size_t)nI * nst * 4 * TR;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % TR);
    const int sh = (int)((e / TR) % 4);
    const size_t bs = e / (4 * TR);             // block * nst + stage
    const int st = (int)(bs % nst), blk = (int)(bs / nst);
    const int I = blk * TR + row;
    const int r0 = st * TK + sh * 4;
    uint32_t w[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float2 x = make_float2(0.f, 0.f);
      if (I < N && r0 + j < R) x = U[(size_t)I * R + r0 + j];
      float rh, rl, ih, il;
      split2(x.x, rh, rl);
      split2(x.y, ih, il);
      w[0][j] = pack_bf16(rh, -ih);
      w[1][j] = pack_bf16(rl, -il);
      w[2][j] = pack_bf16(ih, rh);
      w[3][j] = pack_bf16(il, rl);
    }
    uint32_t* o = out + bs * 4 * WD + lane_off(sh, row);
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<uint4*>(o + (size_t)q * WD) = make_uint4(w[q][0], w[q][1], w[q][2], w[q][3]);
  }
}

// Pair products F_t = conj(psi_occ) psi_unocc of one chunk -> B-side words
// [nT][nst][2][WD] (hi, lo); pairs t >= T and k >= R are zero.  Chunk pair t
// is grid index g = tb + t: occupied row g / nu of po, unoccupied row g % nu of
// pu.  One workgroup covers 128 pairs x 2 stages (32 complex k): it reads both
// rows of every pair as 256-byte segments (16 lanes per row), keeps the
// product in a padded LDS tile, and writes the split words pair-major (64
// lanes = 64 consecutive pairs = 1 KB per store).
constexpr int PP_K = 2 * TK;           // complex k per workgroup
constexpr int PP_PITCH = PP_K + 1;     // complex per LDS row: an odd pitch keeps 32 pair rows on distinct banks

__global__ __launch_bounds__(256) void pair_product_kernel(int R, int nst, int nT, const float2* __restrict__ po,
                                                           const float2* __restrict__ pu, int nu, long tb, int T,
                                                           uint32_t* __restrict__ out) {
  __shared__ float2 F[TR * PP_PITCH];
  const int blk = blockIdx.y;                 // 128-pair block
  const int st0 = blockIdx.x * 2;             // first of two stages
  const int tid = threadIdx.x;
  const int r0 = st0 * TK;
  // phase 1: 16 lanes per pair row, 2 complex (one float4) per lane per pass
  const int sub = tid & 15, prow = tid >> 4;  // 16 pair rows per pass
#pragma unroll
  for (int pass = 0; pass < TR / 16; ++pass) {
    const int p = pass * 16 + prow;
    const int t = blk * TR + p;
    const int r = r0 + 2 * sub;
    float2 f0 = make_float2(0.f, 0.f), f1 = make_float2(0.f, 0.f);
    if (t < T) {
      const long g = tb + t;
      const float2* a = po + (size_t)(g / nu) * R;
      const float2* b = pu + (size_t)(g % nu) * R;
      float2 x0 = make_float2(0.f, 0.f), x1 = x0, y0 = x0, y1 = x0;
      if (r + 1 < R && ((R & 1) == 0)) {
        const float4 xa = *reinterpret_cast<const float4*>(a + r);
        const float4 yb = *reinterpret_cast<const float4*>(b + r);
        x0 = make_float2(xa.x, xa.y); x1 = make_float2(xa.z, xa.w);
        y0 = make_float2(yb.x, yb.y); y1 = make_float2(yb.z, yb.w);
      } else {
        if (r < R) { x0 = a[r]; y0 = b[r]; }
        if (r + 1 < R) { x1 = a[r + 1]; y1 = b[r + 1]; }
      }
      f0 = make_float2(x0.x * y0.x + x0.y * y0.y, x0.x * y0.y - x0.y * y0.x);
      f1 = make_float2(x1.x * y1.x + x1.y * y1.y, x1.x * y1.y - x1.y * y1.x);
    }
    F[p * PP_PITCH + 2 * sub] = f0;
    F[p * PP_PITCH + 2 * sub + 1] = f1;
  }
  __syncthreads();
  // phase 2: lane = pair, 4 complex k per item; 128 pairs x 8 groups per workgroup
#pragma unroll
  for (int it = 0; it < (TR * PP_K / 4) / 256; ++it) {
    const int item = it * 256 + tid;
    const int p = item & (TR - 1), grp = item >> 7;       // grp: 0..7 (stage = grp / 4, sh = grp % 4)
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float2 f = F[p * PP_PITCH + grp * 4 + j];
      float rh, rl, ih, il;
      split2(f.x, rh, rl);
      split2(f.y, ih, il);
      hw[j] = pack_bf16(rh, ih);
      lw[j] = pack_bf16(rl, il);
    }
    const int st = st0 + (grp >> 2);
    if (st < nst) {
      uint32_t* o = out + ((size_t)blk * nst + st) * 2 * WD + lane_off(grp & 3, p);
      *reinterpret_cast<uint4*>(o) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      *reinterpret_cast<uint4*>(o + WD) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
  }
}

// s_j(t) = sqrt(-w_j(t)) with w_j(t) = pair_weight (4 D / (D^2 + omega_j^2),
// D = eps_n - eps_n' < 0, or a spectral-route node share), FP64, zero for the
// padding pairs t in [T, Tp).
__global__ void weights_sqrt_kernel(const double* __restrict__ eps, int n_bands, int n_occ, Chunk c, OmegaList om,
                                    int Tp, float* __restrict__ sw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Tp) return;
  double d = 0.0;
  if (t < c.T) {
    const long g = c.tb + t;
    const int n = c.n0 + (int)(g / c.nu);
    const int u = c.u0 + (int)(g % c.nu);
    d = eps[(size_t)c.k * n_bands + n] - eps[(size_t)c.kq * n_bands + n_occ + u];
  }
  for (int j = 0; j < om.n; ++j) {
    const double w = t < c.T ? pair_weight(d, om, j) : 0.0;
    sw[(size_t)j * Tp + t] = (float)sqrt(fmax(-w, 0.0));
  }
}

// M (tiled complex FP32 [nI][nstT][4][TR][4], written by the projection) ->
// X_j = s_j M as A-side words [n_omega][nIe][nstT][4][WD]: x hi, lo, (-i x) hi, lo.
// Blocks in [nI, nIe) are zero.
__global__ void scale_split_kernel(int nI, int nIe, int nstT, int Tp, int n_omega, const float2* __restrict__ Mt,
                                   const float* __restrict__ sw, uint32_t* __restrict__ X) {
  const size_t total = (size_t)nIe * nstT * 4 * TR;
  const size_t xstride = (size_t)nIe * nstT * 4 * WD;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % TR);
    const int sh = (int)((e / TR) % 4);
    const size_t bs = e / (4 * TR);
    const int st = (int)(bs % nstT), blk = (int)(bs / nstT);
    float2 m[4];
    if (blk < nI) {
      const float4* src = reinterpret_cast<const float4*>(Mt + e * 4);
      const float4 p = src[0], q = src[1];
      m[0] = make_float2(p.x, p.y);
      m[1] = make_float2(p.z, p.w);
      m[2] = make_float2(q.x, q.y);
      m[3] = make_float2(q.z, q.w);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) m[j] = make_float2(0.f, 0.f);
    }
    const int t0 = st * TK + sh * 4;
    uint32_t* o = X + bs * 4 * WD + lane_off(sh, row);
    for (int jw = 0; jw < n_omega; ++jw) {
      const float4 s4 = *reinterpret_cast<const float4*>(sw + (size_t)jw * Tp + t0);
      const float s[4] = {s4.x, s4.y, s4.z, s4.w};
      uint32_t w[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float rh, rl, ih, il;
        split2(s[j] * m[j].x, rh, rl);
        split2(s[j] * m[j].y, ih, il);
        w[0][j] = pack_bf16(rh, ih);
        w[1][j] = pack_bf16(rl, il);
        w[2][j] = pack_bf16(ih, -rh);
        w[3][j] = pack_bf16(il, -rl);
      }
      uint32_t* oj = o + (size_t)jw * xstride;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<uint4*>(oj + (size_t)q * WD) = make_uint4(w[q][0], w[q][1], w[q][2], w[q][3]);
    }
  }
}

// ---- operands of the three-multiplication form
// U (c64 [N][R]) -> plane words [nI][nst][6][HWD]: re hi, lo, im hi, lo,
// (re + im) hi, lo.  Rows >= N and k >= R are zero.  FP16: row I scaled by su[I].
template <int W>
__global__ void tile_u3_kernel(int N, int R, int nI, int nst, const float2* __restrict__ U,
                               const float* __restrict__ su, uint32_t* __restrict__ out) {
  const size_t total = (size_t)nI * nst * 2 * TR;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % TR);
    const int h = (int)((e / TR) % 2);
    const size_t bs = e / (2 * TR);
    const int st = (int)(bs % nst), blk = (int)(bs / nst);
    const int I = blk * TR + row;
    const int r0 = st * TK + 8 * h;
    const float sc = (W == 1 && I < N) ? su[I] : 1.f;
    float re[8], im[8], sm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      float2 x = make_float2(0.f, 0.f);
      if (I < N && r0 + q < R) x = U[(size_t)I * R + r0 + q];
      re[q] = x.x * sc;
      im[q] = x.y * sc;
      sm[q] = (x.x + x.y) * sc;
    }
    uint32_t* o = out + bs * 6 * HWD + lane_off3(h, row);
    uint4 hi, lo;
    pack_plane<W>(re, hi, lo);
    *reinterpret_cast<uint4*>(o) = hi;
    *reinterpret_cast<uint4*>(o + HWD) = lo;
    pack_plane<W>(im, hi, lo);
    *reinterpret_cast<uint4*>(o + 2 * HWD) = hi;
    *reinterpret_cast<uint4*>(o + 3 * HWD) = lo;
    pack_plane<W>(sm, hi, lo);
    *reinterpret_cast<uint4*>(o + 4 * HWD) = hi;
    *reinterpret_cast<uint4*>(o + 5 * HWD) = lo;
  }
}

// Pair products F_t = conj(psi_occ) psi_unocc of one chunk -> plane words
// [nT][nst][6][HWD] (re, im, re + im; hi, lo), pairs t >= T and k >= R zero.
// Same two phases as pair_product_kernel: rows read as 256-byte segments into
// an LDS tile, then lane = pair, 8 k per item, 1 KB per store.
// FP16: pair t scaled by a power of two from the band maxima bmo (rows of po)
// and bmu (rows of pu), |F_t| <= bmo bmu and its planes <= sqrt(2) bmo bmu;
// the scales go to sF[t] (1 past T), written by the first stage-block.
template <int W>
__global__ __launch_bounds__(256) void pair_product3_kernel(int R, int nst, int nT, const float2* __restrict__ po,
                                                            const float2* __restrict__ pu, int nu, long tb, int T,
                                                            const float* __restrict__ bmo,
                                                            const float* __restrict__ bmu, float* __restrict__ sF,
                                                            uint32_t* __restrict__ out) {
  __shared__ float2 F[TR * PP_PITCH];
  const int blk = blockIdx.y;
  const int st0 = blockIdx.x * 2;
  const int tid = threadIdx.x;
  const int r0 = st0 * TK;
  const int sub = tid & 15, prow = tid >> 4;
#pragma unroll
  for (int pass = 0; pass < TR / 16; ++pass) {
    const int p = pass * 16 + prow;
    const int t = blk * TR + p;
    const int r = r0 + 2 * sub;
    float2 f0 = make_float2(0.f, 0.f), f1 = make_float2(0.f, 0.f);
    if (t < T) {
      const long g = tb + t;
      const float2* a = po + (size_t)(g / nu) * R;
      const float2* b = pu + (size_t)(g % nu) * R;
      float2 x0 = make_float2(0.f, 0.f), x1 = x0, y0 = x0, y1 = x0;
      if (r + 1 < R && ((R & 1) == 0)) {
        const float4 xa = *reinterpret_cast<const float4*>(a + r);
        const float4 yb = *reinterpret_cast<const float4*>(b + r);
        x0 = make_float2(xa.x, xa.y); x1 = make_float2(xa.z, xa.w);
        y0 = make_float2(yb.x, yb.y); y1 = make_float2(yb.z, yb.w);
      } else {
        if (r < R) { x0 = a[r]; y0 = b[r]; }
        if (r + 1 < R) { x1 = a[r + 1]; y1 = b[r + 1]; }
      }
      f0 = make_float2(x0.x * y0.x + x0.y * y0.y, x0.x * y0.y - x0.y * y0.x);
      f1 = make_float2(x1.x * y1.x + x1.y * y1.y, x1.x * y1.y - x1.y * y1.x);
    }
    F[p * PP_PITCH + 2 * sub] = f0;
    F[p * PP_PITCH + 2 * sub + 1] = f1;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < (TR * PP_K / 8) / 256; ++it) {
    const int item = it * 256 + tid;
    const int p = item & (TR - 1), grp = item >> 7;   // grp: 0..3 (stage = grp / 2, h = grp % 2)
    float sc = 1.f;
    if constexpr (W == 1) {
      const int t = blk * TR + p;
      if (t < T) {
        const long g = tb + t;
        sc = pow2_scale14(1.41421356f * bmo[g / nu] * bmu[g % nu]);
      }
      if (blockIdx.x == 0 && grp == 0) sF[t] = sc;
    }
    float re[8], im[8], sm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float2 f = F[p * PP_PITCH + grp * 8 + q];
      re[q] = f.x * sc;
      im[q] = f.y * sc;
      sm[q] = (f.x + f.y) * sc;
    }
    const int st = st0 + (grp >> 1);
    if (st < nst) {
      uint32_t* o = out + ((size_t)blk * nst + st) * 6 * HWD + lane_off3(grp & 1, p);
      uint4 hi, lo;
      pack_plane<W>(re, hi, lo);
      *reinterpret_cast<uint4*>(o) = hi;
      *reinterpret_cast<uint4*>(o + HWD) = lo;
      pack_plane<W>(im, hi, lo);
      *reinterpret_cast<uint4*>(o + 2 * HWD) = hi;
      *reinterpret_cast<uint4*>(o + 3 * HWD) = lo;
      pack_plane<W>(sm, hi, lo);
      *reinterpret_cast<uint4*>(o + 4 * HWD) = hi;
      *reinterpret_cast<uint4*>(o + 5 * HWD) = lo;
    }
  }
}

// M (tiled complex FP32, as written by the projection) -> X_j = s_j M as plane
// words [n_omega][nIe][nstT][8][HWD]: a = re x, b = im x, a + b, a - b (hi,
// lo each); the accumulation reads planes 0..5 as its first operand and
// planes 0..3, 6, 7 as the second.  Blocks in [nI, nIe) are zero.
// FP16: row I of frequency j scaled by sX[j * nIe * TR + I].
template <int W>
__global__ void scale_split3_kernel(int nI, int nIe, int nstT, int Tp, int n_omega, const float2* __restrict__ Mt,
                                    const float* __restrict__ sw, const float* __restrict__ sX,
                                    uint32_t* __restrict__ X) {
  const size_t total = (size_t)nIe * nstT * 2 * TR;
  const size_t xstride = (size_t)nIe * nstT * 8 * HWD;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % TR);
    const int h = (int)((e / TR) % 2);
    const size_t bs = e / (2 * TR);
    const int st = (int)(bs % nstT), blk = (int)(bs / nstT);
    float2 m[8];
    if (blk < nI) {
#pragma unroll
      for (int g2 = 0; g2 < 2; ++g2) {
        const float4* src = reinterpret_cast<const float4*>(Mt + ((bs * 4 + 2 * h + g2) * TR + row) * 4);
        const float4 p = src[0], q = src[1];
        m[4 * g2 + 0] = make_float2(p.x, p.y);
        m[4 * g2 + 1] = make_float2(p.z, p.w);
        m[4 * g2 + 2] = make_float2(q.x, q.y);
        m[4 * g2 + 3] = make_float2(q.z, q.w);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) m[q] = make_float2(0.f, 0.f);
    }
    const int t0 = st * TK + 8 * h;
    uint32_t* o = X + bs * 8 * HWD + lane_off3(h, row);
    for (int jw = 0; jw < n_omega; ++jw) {
      const float4 s0 = *reinterpret_cast<const float4*>(sw + (size_t)jw * Tp + t0);
      const float4 s1 = *reinterpret_cast<const float4*>(sw + (size_t)jw * Tp + t0 + 4);
      const float rs = W == 1 ? sX[(size_t)jw * nIe * TR + blk * TR + row] : 1.f;
      const float sv[8] = {s0.x * rs, s0.y * rs, s0.z * rs, s0.w * rs, s1.x * rs, s1.y * rs, s1.z * rs, s1.w * rs};
      float a[8], b[8], ps[8], ms[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = sv[q] * m[q].x;
        b[q] = sv[q] * m[q].y;
        ps[q] = a[q] + b[q];
        ms[q] = a[q] - b[q];
      }
      uint32_t* oj = o + (size_t)jw * xstride;
      uint4 hi, lo;
      pack_plane<W>(a, hi, lo);
      *reinterpret_cast<uint4*>(oj) = hi;
      *reinterpret_cast<uint4*>(oj + HWD) = lo;
      pack_plane<W>(b, hi, lo);
      *reinterpret_cast<uint4*>(oj + 2 * HWD) = hi;
      *reinterpret_cast<uint4*>(oj + 3 * HWD) = lo;
      pack_plane<W>(ps, hi, lo);
      *reinterpret_cast<uint4*>(oj + 4 * HWD) = hi;
      *reinterpret_cast<uint4*>(oj + 5 * HWD) = lo;
      pack_plane<W>(ms, hi, lo);
      *reinterpret_cast<uint4*>(oj + 6 * HWD) = hi;
      *reinterpret_cast<uint4*>(oj + 7 * HWD) = lo;
    }
  }
}

// ---- scales of the FP16 plane words
// su[I] for row I of U: the largest of |re|, |im|, |re + im| over the grid.
__global__ __launch_bounds__(256) void rowscale_u_kernel(int R, const float2* __restrict__ U, float* __restrict__ su) {
  __shared__ float red[256];
  const float2* u = U + (size_t)blockIdx.x * R;
  float m = 0.f;
  for (int r = threadIdx.x; r < R; r += 256) {
    const float2 x = u[r];
    m = fmaxf(m, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fabsf(x.x + x.y)));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) su[blockIdx.x] = pow2_scale14(red[0]);
}

// bm[row] = max over the grid of |psi_row(r)| (one block per band row).
__global__ __launch_bounds__(256) void bandmax_kernel(int R, const float2* __restrict__ psi, float* __restrict__ bm) {
  __shared__ float red[256];
  const float2* p = psi + (size_t)blockIdx.x * R;
  float m = 0.f;
  for (int r = threadIdx.x; r < R; r += 256) {
    const float2 x = p[r];
    m = fmaxf(m, x.x * x.x + x.y * x.y);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) bm[blockIdx.x] = sqrtf(red[0]);
}

// mrow[I] = max over the chunk's pairs of |M_It| (tiled M, one block per row
// block: lane = row, two halves of the stages combined in LDS); rows of the
// padding blocks [nI, nIe) get 0.
__global__ __launch_bounds__(256) void mrow_kernel(int nI, int nstT, const float2* __restrict__ Mt,
                                                   float* __restrict__ mrow) {
  __shared__ float red[256];
  const int blk = blockIdx.x, row = threadIdx.x & (TR - 1), half = threadIdx.x >> 7;
  float m = 0.f;
  if (blk < nI)
    for (int st = half; st < nstT; st += 2)
#pragma unroll
      for (int sh = 0; sh < 4; ++sh) {
        const float4* src = reinterpret_cast<const float4*>(Mt + ((((size_t)blk * nstT + st) * 4 + sh) * TR + row) * 4);
        const float4 a = src[0], b = src[1];
        m = fmaxf(m, fmaxf(fmaxf(a.x * a.x + a.y * a.y, a.z * a.z + a.w * a.w),
                           fmaxf(b.x * b.x + b.y * b.y, b.z * b.z + b.w * b.w)));
      }
  red[threadIdx.x] = m;
  __syncthreads();
  if (half == 0) mrow[blk * TR + row] = sqrtf(fmaxf(red[row], red[row + TR]));
}

// sX[j][I] for the scaled operands X_j = s_j M: the bound sqrt(2) max_t |M_It|
// max_t s_j(t) of their planes (a, b, a + b, a - b).
__global__ __launch_bounds__(256) void xscale_kernel(int rows, int Tp, const float* __restrict__ sw,
                                                     const float* __restrict__ mrow, float* __restrict__ sX) {
  __shared__ float red[256];
  const int j = blockIdx.x;
  float m = 0.f;
  for (int t = threadIdx.x; t < Tp; t += 256) m = fmaxf(m, sw[(size_t)j * Tp + t]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const float smax = red[0];
  for (int I = threadIdx.x; I < rows; I += 256) sX[(size_t)j * rows + I] = pow2_scale14(1.41421356f * mrow[I] * smax);
}

// W^c_j = W_j - diag(v) (c128 [N][N]) -> A-side words [nI][nstN][4][WD]
// (conj hi, lo, swap hi, lo), zero outside N x N.
__global__ void tile_wc_kernel(int N, int nI, int nst, const double2* __restrict__ W, const double* __restrict__ v,
                               uint32_t* __restrict__ out) {
  const size_t total = (size_t)nI * nst * 4 * TR;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % TR);
    const int sh = (int)((e / TR) % 4);
    const size_t bs = e / (4 * TR);
    const int st = (int)(bs % nst), blk = (int)(bs / nst);
    const int I = blk * TR + row;
    const int c0 = st * TK + sh * 4;
    uint32_t w[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double2 x = make_double2(0.0, 0.0);
      const int c = c0 + j;
      if (I < N && c < N) {
        x = W[(size_t)I * N + c];
        if (c == I) x.x -= v[I];
      }
      float rh, rl, ih, il;
      split2((float)x.x, rh, rl);
      split2((float)x.y, ih, il);
      w[0][j] = pack_bf16(rh, -ih);
      w[1][j] = pack_bf16(rl, -il);
      w[2][j] = pack_bf16(ih, rh);
      w[3][j] = pack_bf16(il, rl);
    }
    uint32_t* o = out + bs * 4 * WD + lane_off(sh, row);
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<uint4*>(o + (size_t)q * WD) = make_uint4(w[q][0], w[q][1], w[q][2], w[q][3]);
  }
}

// Columns of M (c64 rows [N][ldm], columns < nb valid) -> B-side words
// [nb_pad/128][nstN][2][WD] with the reduction index running over the rows of
// M (hi, lo); zero for columns >= nb and rows >= N.
__global__ void tile_cols_kernel(int N, int nb, int nTb, int nst, const float2* __restrict__ M, long ldm,
                                 uint32_t* __restrict__ out) {
  const size_t total = (size_t)nTb * nst * 4 * TR;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(e % TR);
    const int sh = (int)((e / TR) % 4);
    const size_t bs = e / (4 * TR);
    const int st = (int)(bs % nst), blk = (int)(bs / nst);
    const int c = blk * TR + col;
    const int r0 = st * TK + sh * 4;
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float2 x = make_float2(0.f, 0.f);
      if (c < nb && r0 + j < N) x = M[(size_t)(r0 + j) * ldm + c];
      float rh, rl, ih, il;
      split2(x.x, rh, rl);
      split2(x.y, ih, il);
      hw[j] = pack_bf16(rh, ih);
      lw[j] = pack_bf16(rl, il);
    }
    uint32_t* o = out + bs * 2 * WD + lane_off(sh, col);
    *reinterpret_cast<uint4*>(o) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    *reinterpret_cast<uint4*>(o + WD) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
  }
}

// Operands of the self-energy's W^c M products for the three-multiplication
// core.  W^c = W - diag(v) (c128 [N][N]) -> plane words [nI][nstN][6][HWD]:
// re, im, re + im (hi, lo) of row I, k running over the columns of W^c;
// zero for rows or columns >= N.
__global__ void tile_wc3_kernel(int N, int nI, int nst, const double2* __restrict__ W, const double* __restrict__ v,
                                uint32_t* __restrict__ out) {
  const size_t total = (size_t)nI * nst * 2 * TR;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % TR);
    const int h = (int)((e / TR) % 2);
    const size_t bs = e / (2 * TR);
    const int st = (int)(bs % nst), blk = (int)(bs / nst);
    const int I = blk * TR + row;
    const int c0 = st * TK + 8 * h;
    float re[8], im[8], sm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double2 x = make_double2(0.0, 0.0);
      const int c = c0 + q;
      if (I < N && c < N) {
        x = W[(size_t)I * N + c];
        if (c == I) x.x -= v[I];
      }
      re[q] = (float)x.x;
      im[q] = (float)x.y;
      sm[q] = re[q] + im[q];
    }
    uint32_t* o = out + bs * 6 * HWD + lane_off3(h, row);
    uint4 hi, lo;
    pack_plane<0>(re, hi, lo);
    *reinterpret_cast<uint4*>(o) = hi;
    *reinterpret_cast<uint4*>(o + HWD) = lo;
    pack_plane<0>(im, hi, lo);
    *reinterpret_cast<uint4*>(o + 2 * HWD) = hi;
    *reinterpret_cast<uint4*>(o + 3 * HWD) = lo;
    pack_plane<0>(sm, hi, lo);
    *reinterpret_cast<uint4*>(o + 4 * HWD) = hi;
    *reinterpret_cast<uint4*>(o + 5 * HWD) = lo;
  }
}

// Columns of M (c64 rows [N][ldm], columns < nb valid) -> plane words
// [nb_pad/128][nstN][6][HWD] (re, im, re + im; hi, lo) with k running over the
// rows of M; zero for columns >= nb and rows >= N.
__global__ void tile_cols3_kernel(int N, int nb, int nTb, int nst, const float2* __restrict__ M, long ldm,
                                  uint32_t* __restrict__ out) {
  const size_t total = (size_t)nTb * nst * 2 * TR;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(e % TR);
    const int h = (int)((e / TR) % 2);
    const size_t bs = e / (2 * TR);
    const int st = (int)(bs % nst), blk = (int)(bs / nst);
    const int c = blk * TR + col;
    const int r0 = st * TK + 8 * h;
    float re[8], im[8], sm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      float2 x = make_float2(0.f, 0.f);
      if (c < nb && r0 + q < N) x = M[(size_t)(r0 + q) * ldm + c];
      re[q] = x.x;
      im[q] = x.y;
      sm[q] = x.x + x.y;
    }
    uint32_t* o = out + bs * 6 * HWD + lane_off3(h, col);
    uint4 hi, lo;
    pack_plane<0>(re, hi, lo);
    *reinterpret_cast<uint4*>(o) = hi;
    *reinterpret_cast<uint4*>(o + HWD) = lo;
    pack_plane<0>(im, hi, lo);
    *reinterpret_cast<uint4*>(o + 2 * HWD) = hi;
    *reinterpret_cast<uint4*>(o + 3 * HWD) = lo;
    pack_plane<0>(sm, hi, lo);
    *reinterpret_cast<uint4*>(o + 4 * HWD) = hi;
    *reinterpret_cast<uint4*>(o + 5 * HWD) = lo;
  }
}

// q[n'] = Re sum_mu conj(M[mu][n']) Y[mu][n'] in two fixed-order passes: a
// workgroup covers 32 columns and one chunk of rows (8 row groups of 32
// lanes, combined in LDS), then the chunks are summed in order.
constexpr int CD_CHUNKS = 16;

__global__ __launch_bounds__(256) void coldot_f32_kernel(int N, int nb, const float2* __restrict__ M,
                                                         const float2* __restrict__ Y, long ld, int rows_per_chunk,
                                                         double* __restrict__ part) {
  __shared__ double red[8][32];
  const int cx = threadIdx.x & 31, ry = threadIdx.x >> 5;
  const int c = blockIdx.x * 32 + cx;
  const int r0 = blockIdx.y * rows_per_chunk, r1 = min(N, r0 + rows_per_chunk);
  double acc = 0.0;
  if (c < nb)
    for (int r = r0 + ry; r < r1; r += 8) {
      const float2 m = M[(size_t)r * ld + c], y = Y[(size_t)r * ld + c];
      acc += (double)m.x * (double)y.x + (double)m.y * (double)y.y;
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

__global__ void coldot_reduce_kernel(int nb, int chunks, const double* __restrict__ part, double* __restrict__ q) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nb) return;
  double t = 0.0;
  for (int k = 0; k < chunks; ++k) t += part[(size_t)k * nb + c];
  q[c] = t;
}

// ------------------------------------------- real operands (inversion symmetry)
// With real U and real wave functions every product is real: one word holds
// two consecutive real k values, a block-stage covers 32 k, and the operands
// need only hi and lo (no sign or swap patterns).
__device__ inline void split_pair(float a, float b, uint32_t& hi, uint32_t& lo) {
  float ah, al, bh, bl;
  split2(a, ah, al);
  split2(b, bh, bl);
  hi = pack_bf16(ah, bh);
  lo = pack_bf16(al, bl);
}

// U (float [N][R]) -> A-side words [nI][nst][2][WD] (hi, lo), zero outside.
__global__ void tile_u_real_kernel(int N, int R, int nI, int nst, const float* __restrict__ U,
                                   uint32_t* __restrict__ out) {
  const size_t total = (size_t)nI * nst * 4 * TR;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % TR);
    const int sh = (int)((e / TR) % 4);
    const size_t bs = e / (4 * TR);
    const int st = (int)(bs % nst), blk = (int)(bs / nst);
    const int I = blk * TR + row;
    const int r0 = st * 2 * TK + sh * 8;
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + 2 * j;
      const float a = (I < N && r < R) ? U[(size_t)I * R + r] : 0.f;
      const float b = (I < N && r + 1 < R) ? U[(size_t)I * R + r + 1] : 0.f;
      split_pair(a, b, hw[j], lw[j]);
    }
    uint32_t* o = out + bs * 2 * WD + lane_off(sh, row);
    *reinterpret_cast<uint4*>(o) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    *reinterpret_cast<uint4*>(o + WD) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
  }
}

// Real pair products F_t = psi_n psi_n' -> B-side words [nT][nst][2][WD]
// (pairs t >= T and k >= R zero).  Same two phases as the complex kernels: a
// workgroup takes 128 pairs x 64 real k (two block-stages); 16 lanes read
// each pair's two rows as 256-byte segments into an LDS tile, then lane =
// pair, 8 k per item, 1 KB per store.
constexpr int PPR_K = 4 * TK;              // real k per workgroup
constexpr int PPR_PITCH = PPR_K + 1;       // odd pitch: 32 pair rows on distinct banks
__global__ __launch_bounds__(256) void pair_product_real_kernel(int R, int nst, int nT, const float* __restrict__ po,
                                                                const float* __restrict__ pu, int nu, long tb, int T,
                                                                uint32_t* __restrict__ out) {
  __shared__ float F[TR * PPR_PITCH];
  const int blk = blockIdx.y;
  const int st0 = blockIdx.x * 2;
  const int tid = threadIdx.x;
  const int r0 = st0 * 2 * TK;
  const int sub = tid & 15, prow = tid >> 4;
#pragma unroll
  for (int pass = 0; pass < TR / 16; ++pass) {
    const int p = pass * 16 + prow;
    const int t = blk * TR + p;
    const int r = r0 + 4 * sub;
    float f[4] = {0.f, 0.f, 0.f, 0.f};
    if (t < T) {
      const long g = tb + t;
      const float* a = po + (size_t)(g / nu) * R;
      const float* b = pu + (size_t)(g % nu) * R;
      if (r + 3 < R && (R & 3) == 0) {
        const float4 x = *reinterpret_cast<const float4*>(a + r);
        const float4 y = *reinterpret_cast<const float4*>(b + r);
        f[0] = x.x * y.x; f[1] = x.y * y.y; f[2] = x.z * y.z; f[3] = x.w * y.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (r + j < R) f[j] = a[r + j] * b[r + j];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) F[p * PPR_PITCH + 4 * sub + j] = f[j];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < (TR * PPR_K / 8) / 256; ++it) {
    const int item = it * 256 + tid;
    const int p = item & (TR - 1), grp = item >> 7;   // grp 0..7: stage st0 + grp / 4, sub-half grp % 4
    const int st = st0 + (grp >> 2);
    if (st < nst) {
      uint32_t hw[4], lw[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        split_pair(F[p * PPR_PITCH + grp * 8 + 2 * j], F[p * PPR_PITCH + grp * 8 + 2 * j + 1], hw[j], lw[j]);
      uint32_t* o = out + ((size_t)blk * nst + st) * 2 * WD + lane_off(grp & 3, p);
      *reinterpret_cast<uint4*>(o) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      *reinterpret_cast<uint4*>(o + WD) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
  }
}

// Real M (tiled [nI][nstT][4][TR][8] floats) -> X_j = s_j M as words
// [n_omega][nIe][nstT][2][WD] (hi, lo); blocks in [nI, nIe) are zero.
__global__ void scale_split_real_kernel(int nI, int nIe, int nstT, int Tp, int n_omega, const float* __restrict__ Mt,
                                        const float* __restrict__ sw, uint32_t* __restrict__ X) {
  const size_t total = (size_t)nIe * nstT * 4 * TR;
  const size_t xstride = (size_t)nIe * nstT * 2 * WD;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % TR);
    const int sh = (int)((e / TR) % 4);
    const size_t bs = e / (4 * TR);
    const int st = (int)(bs % nstT), blk = (int)(bs / nstT);
    float m[8];
    if (blk < nI) {
      const float4* src = reinterpret_cast<const float4*>(Mt + e * 8);
      const float4 p = src[0], q = src[1];
      m[0] = p.x; m[1] = p.y; m[2] = p.z; m[3] = p.w; m[4] = q.x; m[5] = q.y; m[6] = q.z; m[7] = q.w;
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) m[j] = 0.f;
    }
    const int t0 = st * 2 * TK + sh * 8;
    uint32_t* o = X + bs * 2 * WD + lane_off(sh, row);
    for (int jw = 0; jw < n_omega; ++jw) {
      const float4 s0 = *reinterpret_cast<const float4*>(sw + (size_t)jw * Tp + t0);
      const float4 s1 = *reinterpret_cast<const float4*>(sw + (size_t)jw * Tp + t0 + 4);
      const float sc[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
      uint32_t hw[4], lw[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) split_pair(sc[2 * j] * m[2 * j], sc[2 * j + 1] * m[2 * j + 1], hw[j], lw[j]);
      uint32_t* oj = o + (size_t)jw * xstride;
      *reinterpret_cast<uint4*>(oj) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      *reinterpret_cast<uint4*>(oj + WD) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
  }
}

// --------------------------------------------------------------- GEMM core

// Workgroups are handed to the 8 XCDs round-robin by linear id; renumber them
// so that each XCD works through one contiguous range of tiles (neighbouring
// tiles share operand blocks in that XCD's L2).
__device__ inline int xcd_remap(int L, int G) {
  const int base = G / 8, rem = G % 8;
  const int x = L % 8, local = L / 8;
  return x < rem ? x * (base + 1) + local : rem * (base + 1) + (x - rem) * base + local;
}

// Lower tiles (128-row block ti, 256-col block bj, ti >= 2 bj) in groups of
// eight row blocks, column block by column block inside a group.
__device__ inline void lower_tile_grouped(int l, int nI, int& ti, int& bj) {
  for (int t0 = 0; t0 < nI; t0 += 8) {
    const int t1 = min(t0 + 8, nI);
    const int bjmax = (t1 - 1) / 2;
    for (int b = 0; b <= bjmax; ++b) {
      const int lo = max(t0, 2 * b);
      const int cnt = t1 - lo;
      if (l < cnt) {
        ti = lo + l;
        bj = b;
        return;
      }
      l -= cnt;
    }
  }
  ti = 0;
  bj = 0;
}

enum GemmOut { OUT_TILED = 0, OUT_ROWS = 1, OUT_HERK = 2 };

struct GemmArgs {
  const uint32_t* A;   // A-side words, 4 per block-stage
  const uint32_t* B;   // B-side words, first two of b_words per block-stage
  int b_words;
  size_t a_bstride;    // dwords between consecutive row blocks of A
  size_t b_bstride;    // dwords between consecutive column blocks of B
  int nst;             // stages (K / 16)
  size_t omega_stride; // dwords between frequencies of A and B (accumulation)
  int nI;              // row blocks of A
  int nTj;             // 256-col tiles (projection)
  int n_tiles;         // lower tiles per frequency (accumulation)
  int N, T;            // valid rows / cols
  float2* M;           // OUT_TILED: [nI][nst_out][4][TR][4]; OUT_ROWS: [N][ldm]
  long ldm;
  int nst_out;
  double2* P;          // OUT_HERK: n_omega x [N][N]
  // three-multiplication core only: plane words per block-stage of A and B,
  // the plane of B holding c + d (projection) or c - d (accumulation), and
  // the sign s of Re = T1 + s T2, Im = T3 - T1 + s T2
  int a_words3, b_words3, b_sum3;
  float sigma3;
  // FP16 plane words: scales of the A rows and B columns (projection), or of
  // the rows of frequency jw at sa + jw * s_stride (accumulation, both sides)
  const float* sa;
  const float* sb;
  size_t s_stride;
};

__device__ inline floatx16 mma(uint4 a, uint4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// One stage of operands in flight through registers: A 32 KB, B two 16 KB
// halves (named members: arrays of vectors here end up in scratch memory).
struct Staged {
  uint4 a0, a1, a2, a3, a4, a5, a6, a7, b0, b1, b2, b3, c0, c1, c2, c3;
};

__device__ __forceinline__ uint4 ld16(const uint32_t* p, int q, int tid) {
  return *reinterpret_cast<const uint4*>(p + (q * GT + tid) * 4);
}
__device__ __forceinline__ void st16(uint32_t* p, int q, int tid, uint4 v) {
  *reinterpret_cast<uint4*>(p + (q * GT + tid) * 4) = v;
}

__device__ __forceinline__ void stage_load(Staged& r, const uint32_t* Ap, const uint32_t* B0, const uint32_t* B1,
                                           size_t b_step, int st, int tid) {
  const uint32_t* a = Ap + (size_t)st * 4 * WD;
  const uint32_t* b0 = B0 + (size_t)st * b_step;
  const uint32_t* b1 = B1 + (size_t)st * b_step;
  r.a0 = ld16(a, 0, tid); r.a1 = ld16(a, 1, tid); r.a2 = ld16(a, 2, tid); r.a3 = ld16(a, 3, tid);
  r.a4 = ld16(a, 4, tid); r.a5 = ld16(a, 5, tid); r.a6 = ld16(a, 6, tid); r.a7 = ld16(a, 7, tid);
  r.b0 = ld16(b0, 0, tid); r.b1 = ld16(b0, 1, tid); r.b2 = ld16(b0, 2, tid); r.b3 = ld16(b0, 3, tid);
  r.c0 = ld16(b1, 0, tid); r.c1 = ld16(b1, 1, tid); r.c2 = ld16(b1, 2, tid); r.c3 = ld16(b1, 3, tid);
}

// LDS stage: A words at [0, 4 WD), B half c word q at 4 WD + (2 c + q) WD.
// part 0 stores A, part 1 stores B.
__device__ __forceinline__ void stage_store(const Staged& r, uint32_t* L, int part, int tid) {
  if (part == 0) {
    st16(L, 0, tid, r.a0); st16(L, 1, tid, r.a1); st16(L, 2, tid, r.a2); st16(L, 3, tid, r.a3);
    st16(L, 4, tid, r.a4); st16(L, 5, tid, r.a5); st16(L, 6, tid, r.a6); st16(L, 7, tid, r.a7);
  } else {
    uint32_t* b0 = L + 4 * WD;
    uint32_t* b1 = L + 6 * WD;
    st16(b0, 0, tid, r.b0); st16(b0, 1, tid, r.b1); st16(b0, 2, tid, r.b2); st16(b0, 3, tid, r.b3);
    st16(b1, 0, tid, r.c0); st16(b1, 1, tid, r.c1); st16(b1, 2, tid, r.c2); st16(b1, 3, tid, r.c3);
  }
}

struct Frags {
  uint4 a[4][2];   // A words (conj|x hi, lo, swap|-ix hi, lo) x row blocks
  uint4 b[2][4];   // B words (hi, lo) x column blocks
};

__device__ __forceinline__ void read_frags(Frags& f, const uint32_t* L, int s, int wm, int wn, int l32, int h) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
      f.a[q][rb] = *reinterpret_cast<const uint4*>(L + q * WD + lane_off(s * 2 + h, wm * 64 + rb * 32 + l32));
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
      f.b[q][cb] = *reinterpret_cast<const uint4*>(L + (4 + 2 * wn + q) * WD + lane_off(s * 2 + h, cb * 32 + l32));
}

// 48 MFMAs: re += A0h Bh + A0h Bl + A0l Bh, im likewise with A1.
__device__ __forceinline__ void mma_step(const Frags& f, floatx16 (&cr)[2][4], floatx16 (&ci)[2][4]) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      cr[rb][cb] = mma(f.a[0][rb], f.b[0][cb], cr[rb][cb]);
      ci[rb][cb] = mma(f.a[2][rb], f.b[0][cb], ci[rb][cb]);
      cr[rb][cb] = mma(f.a[0][rb], f.b[1][cb], cr[rb][cb]);
      ci[rb][cb] = mma(f.a[2][rb], f.b[1][cb], ci[rb][cb]);
      cr[rb][cb] = mma(f.a[1][rb], f.b[0][cb], cr[rb][cb]);
      ci[rb][cb] = mma(f.a[3][rb], f.b[0][cb], ci[rb][cb]);
    }
}

// The 24 MFMAs of mma_step for row block rb.
__device__ __forceinline__ void mma_half(const Frags& f, int rb, floatx16 (&cr)[2][4], floatx16 (&ci)[2][4]) {
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    cr[rb][cb] = mma(f.a[0][rb], f.b[0][cb], cr[rb][cb]);
    ci[rb][cb] = mma(f.a[2][rb], f.b[0][cb], ci[rb][cb]);
    cr[rb][cb] = mma(f.a[0][rb], f.b[1][cb], cr[rb][cb]);
    ci[rb][cb] = mma(f.a[2][rb], f.b[1][cb], ci[rb][cb]);
    cr[rb][cb] = mma(f.a[1][rb], f.b[0][cb], cr[rb][cb]);
    ci[rb][cb] = mma(f.a[3][rb], f.b[0][cb], ci[rb][cb]);
  }
}

// Scheduling-group masks (LLVM AMDGPU): MFMA, global load, LDS read, LDS write.
constexpr int SG_MFMA = 0x008, SG_VMR = 0x020, SG_DSR = 0x100, SG_DSW = 0x200;

// Workgroup barrier ordering LDS only (global loads in flight stay in flight).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One K stage (two MFMA steps of 8 complex k) from LDS buffer st % 2; r holds
// stage st + 1 on entry and stage st + 2 on exit.  The order is pinned:
//   fragments of step 0;
//   step 0 MFMAs with r written to the idle buffer and the fragments of
//   step 1 read between them;
//   global loads of stage st + 2 into r, then step 1 MFMAs.
__device__ __forceinline__ void mma_stage(uint32_t* lds, int st, Staged& r, const uint32_t* Ap, const uint32_t* B0,
                                          const uint32_t* B1, size_t b_step, int nst, int tid, int wm, int wn,
                                          int l32, int h, floatx16 (&cr)[2][4], floatx16 (&ci)[2][4]) {
  const uint32_t* L = lds + (st & 1) * LDS_STAGE;
  uint32_t* Ln = lds + ((st + 1) & 1) * LDS_STAGE;
  Frags f0, f1;
  read_frags(f0, L, 0, wm, wn, l32, h);
  __builtin_amdgcn_sched_barrier(0);
  stage_store(r, Ln, 0, tid);
  stage_store(r, Ln, 1, tid);
  read_frags(f1, L, 1, wm, wn, l32, h);
  mma_step(f0, cr, ci);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
    __builtin_amdgcn_sched_group_barrier(SG_DSW, 1, 0);
    __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
    __builtin_amdgcn_sched_group_barrier(SG_DSR, 1, 0);
    __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
  }
  __builtin_amdgcn_sched_barrier(0);
  stage_load(r, Ap, B0, B1, b_step, min(st + 2, nst - 1), tid);
  mma_step(f1, cr, ci);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    __builtin_amdgcn_sched_group_barrier(SG_VMR, 1, 0);
    __builtin_amdgcn_sched_group_barrier(SG_MFMA, 3, 0);
  }
  __builtin_amdgcn_sched_barrier(0);
}

typedef __attribute__((address_space(3))) void lds_void;

// Direct global -> LDS copy of one stage (global_load_lds_dwordx4): lane i of
// a wave writes the 16 bytes at the wave's (uniform) LDS address + 16 i, so
// the tiled operand image lands in LDS exactly as it lies in memory.
__device__ __forceinline__ void stage_dma(uint32_t* Ln, const uint32_t* Ap, const uint32_t* B0, const uint32_t* B1,
                                          size_t b_step, int st, int tid, int w) {
  const uint32_t* a = Ap + (size_t)st * 4 * WD;
  const uint32_t* b0 = B0 + (size_t)st * b_step;
  const uint32_t* b1 = B1 + (size_t)st * b_step;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    __builtin_amdgcn_global_load_lds(a + (q * GT + tid) * 4, (lds_void*)(Ln + (q * GT + w * 64) * 4), 16, 0, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    __builtin_amdgcn_global_load_lds(b0 + (q * GT + tid) * 4, (lds_void*)(Ln + 4 * WD + (q * GT + w * 64) * 4), 16,
                                     0, 0);
    __builtin_amdgcn_global_load_lds(b1 + (q * GT + tid) * 4, (lds_void*)(Ln + 6 * WD + (q * GT + w * 64) * 4), 16,
                                     0, 0);
  }
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima).
__device__ __forceinline__ void wait_vm0() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// One K stage with direct-to-LDS staging: all fragments of the stage are
// read first (a copy into LDS makes every later LDS read wait for it), the
// first 24 MFMAs start, then the copy of stage st + 1 into the idle buffer
// is issued and has the remaining 72 MFMAs to land.
__device__ __forceinline__ void mma_stage_dma(uint32_t* lds, int st, const uint32_t* Ap, const uint32_t* B0,
                                              const uint32_t* B1, size_t b_step, int nst, int tid, int w, int wm,
                                              int wn, int l32, int h, floatx16 (&cr)[2][4], floatx16 (&ci)[2][4]) {
  const uint32_t* L = lds + (st & 1) * LDS_STAGE;
  uint32_t* Ln = lds + ((st + 1) & 1) * LDS_STAGE;
  Frags f0, f1;
  read_frags(f0, L, 0, wm, wn, l32, h);
  read_frags(f1, L, 1, wm, wn, l32, h);
  mma_half(f0, 0, cr, ci);
  __builtin_amdgcn_sched_barrier(0);
  if (st + 1 < nst) stage_dma(Ln, Ap, B0, B1, b_step, st + 1, tid, w);
  __builtin_amdgcn_sched_barrier(0);
  mma_half(f0, 1, cr, ci);
  mma_step(f1, cr, ci);
  __builtin_amdgcn_sched_barrier(0);
}

// Output tile of this workgroup: row block ti (128 rows), column tile tj
// (256 columns) and, for the accumulation, frequency jw.
template <int OUT>
__device__ __forceinline__ void decode_tile(const GemmArgs& g, int& ti, int& tj, int& jw) {
  const int V = xcd_remap(blockIdx.x, gridDim.x);
  jw = 0;
  if constexpr (OUT == OUT_HERK) {
    jw = V / g.n_tiles;
    lower_tile_grouped(V % g.n_tiles, g.nI, ti, tj);
  } else {
    const int per = 8 * g.nTj;
    const int grp = V / per, within = V % per;
    const int gsz = min(8, g.nI - grp * 8);
    tj = within / gsz;
    ti = grp * 8 + within % gsz;
  }
}

template <int OUT, int DMA>
__global__ __launch_bounds__(GT, 1) void gemm_bf16x3_kernel(GemmArgs g) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  int ti, tj, jw;
  decode_tile<OUT>(g, ti, tj, jw);
  const uint32_t* Ap = g.A + jw * g.omega_stride + ti * g.a_bstride;
  const uint32_t* B0 = g.B + jw * g.omega_stride + (size_t)(2 * tj) * g.b_bstride;
  const uint32_t* B1 = B0 + g.b_bstride;
  const size_t b_step = (size_t)g.b_words * WD;

  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = w >> 1, wn = w & 1;
  const int l32 = lane & 31, h = lane >> 5;

  floatx16 cr[2][4], ci[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        cr[a][b][v] = 0.f;
        ci[a][b][v] = 0.f;
      }

  if constexpr (DMA) {
    stage_dma(lds, Ap, B0, B1, b_step, 0, tid, w);
    wait_vm0();
    lds_barrier();
    for (int st = 0; st < g.nst; ++st) {
      mma_stage_dma(lds, st, Ap, B0, B1, b_step, g.nst, tid, w, wm, wn, l32, h, cr, ci);
      wait_vm0();
      lds_barrier();
    }
  } else {
    // The staged registers hold the next stage while the current one is
    // multiplied from LDS; they are written to the idle buffer early in the
    // iteration and then receive the stage after next, so each global load
    // has about one iteration to arrive.
    Staged r;
    stage_load(r, Ap, B0, B1, b_step, 0, tid);
    stage_store(r, lds, 0, tid);
    stage_store(r, lds, 1, tid);
    stage_load(r, Ap, B0, B1, b_step, min(1, g.nst - 1), tid);
    lds_barrier();
    // (past the end, loads repeat the final stage, in bounds, and stores fill
    // the idle buffer, which is never read)
    for (int st = 0; st < g.nst; ++st) {
      mma_stage(lds, st, r, Ap, B0, B1, b_step, g.nst, tid, wm, wn, l32, h, cr, ci);
      lds_barrier();
    }
  }

  if constexpr (OUT == OUT_HERK) {
    // P_j -= C over the lower triangle in FP64.  The FP32 tile goes through
    // LDS in two 128-column halves so that the read-modify-write of P runs
    // as a short loop over coalesced rows (FP64 conversions of the whole
    // register tile at once would not fit in registers).
    float2* E = reinterpret_cast<float2*>(lds);   // [128][128]
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (wn == c) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
              E[row * 128 + cb * 32 + l32] = make_float2(cr[rb][cb][v], ci[rb][cb][v]);
            }
      }
      __syncthreads();
      double2* Pj = g.P + (size_t)jw * g.N * g.N;
#pragma unroll 4
      for (int e = tid; e < 128 * 128; e += GT) {
        const int gi = ti * TM + (e >> 7), gj = tj * TN + c * 128 + (e & 127);
        if (gi < g.N && gj <= gi) {
          const float2 x = E[e];
          double2* p = Pj + (size_t)gi * g.N + gj;
          double2 y = *p;
          y.x -= (double)x.x;
          y.y -= (double)x.y;
          *p = y;
        }
      }
      __syncthreads();
    }
    return;
  }
  // epilogue: element (row, col) of block (rb, cb), register v
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * 128 + cb * 32 + l32;
        const float re = cr[rb][cb][v], im = ci[rb][cb][v];
        if constexpr (OUT == OUT_TILED) {
          const int t = tj * TN + col;
          const size_t bs = (size_t)ti * g.nst_out + t / TK;
          const int kk = t % TK;
          g.M[(bs * 4 + (kk >> 2)) * TR * 4 + row * 4 + (kk & 3)] = make_float2(re, im);
        } else {
          const int gi = ti * TM + row, gt = tj * TN + col;
          if (gi < g.N && gt < g.T) g.M[(size_t)gi * g.ldm + gt] = make_float2(re, im);
        }
      }
}

// ---------------------------------------------- 8-wave variant of the core
// Same tile (128 x 256), operands, LDS image and epilogues, with 8 waves (two
// per SIMD) of 64 x 64 outputs each (128 accumulators per lane), so that one
// wave's waits on LDS, barriers and loads overlap the other wave's MFMAs.
constexpr int GT8 = 512;

// AW A-side words per block-stage: 4 for complex operands (conj|x, swap|-ix;
// hi, lo), 2 for real ones (hi, lo; a dword then holds two consecutive real
// k values, so a block-stage covers 32 real k).
template <int AW>
struct Staged8 {
  uint4 a[AW];
  uint4 b0, b1, c0, c1;
};

template <int AW>
__device__ __forceinline__ void stage_load8(Staged8<AW>& r, const uint32_t* Ap, const uint32_t* B0,
                                            const uint32_t* B1, size_t b_step, int st, int tid) {
  const uint32_t* a = Ap + (size_t)st * AW * WD;
  const uint32_t* b0 = B0 + (size_t)st * b_step;
  const uint32_t* b1 = B1 + (size_t)st * b_step;
  auto ld = [&](const uint32_t* p, int q) __attribute__((always_inline)) {
    return *reinterpret_cast<const uint4*>(p + (q * GT8 + tid) * 4);
  };
#pragma unroll
  for (int q = 0; q < AW; ++q) r.a[q] = ld(a, q);
  r.b0 = ld(b0, 0); r.b1 = ld(b0, 1); r.c0 = ld(b1, 0); r.c1 = ld(b1, 1);
}

// LDS stage: A words at [0, AW WD), B half c word q at (AW + 2 c + q) WD.
template <int AW>
__device__ __forceinline__ void stage_store8(const Staged8<AW>& r, uint32_t* L, int part, int tid) {
  auto st = [&](uint32_t* p, int q, uint4 v) __attribute__((always_inline)) {
    *reinterpret_cast<uint4*>(p + (q * GT8 + tid) * 4) = v;
  };
  if (part == 0) {
#pragma unroll
    for (int q = 0; q < AW; ++q) st(L, q, r.a[q]);
  } else {
    st(L + AW * WD, 0, r.b0); st(L + AW * WD, 1, r.b1); st(L + (AW + 2) * WD, 0, r.c0); st(L + (AW + 2) * WD, 1, r.c1);
  }
}

template <int AW>
struct Frags8 {
  uint4 a[AW][2];
  uint4 b[2][2];
};

template <bool REAL>
constexpr size_t gemm8_lds_bytes() {
  return 2 * (size_t)((REAL ? 2 : 4) + 4) * WD * sizeof(uint32_t);
}

template <int OUT, bool REAL = false>
__global__ __launch_bounds__(GT8, 1) void gemm8_bf16x3_kernel(GemmArgs g) {
  constexpr int AW = REAL ? 2 : 4;
  constexpr int STAGE = (AW + 4) * WD;
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  int ti, tj, jw;
  decode_tile<OUT>(g, ti, tj, jw);
  const uint32_t* Ap = g.A + jw * g.omega_stride + ti * g.a_bstride;
  const uint32_t* B0 = g.B + jw * g.omega_stride + (size_t)(2 * tj) * g.b_bstride;
  const uint32_t* B1 = B0 + g.b_bstride;
  const size_t b_step = (size_t)g.b_words * WD;

  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = w >> 2, wn = w & 3;          // rows wm*64, columns wn*64
  const int half = wn >> 1, c0 = (wn & 1) * 64;  // B half holding this wave's columns
  const int l32 = lane & 31, h = lane >> 5;

  floatx16 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        cr[a][b][v] = 0.f;
        ci[a][b][v] = 0.f;
      }

  Staged8<AW> r;
  stage_load8<AW>(r, Ap, B0, B1, b_step, 0, tid);
  stage_store8<AW>(r, lds, 0, tid);
  stage_store8<AW>(r, lds, 1, tid);
  stage_load8<AW>(r, Ap, B0, B1, b_step, min(1, g.nst - 1), tid);
  lds_barrier();
  for (int st = 0; st < g.nst; ++st) {
    const uint32_t* L = lds + (st & 1) * STAGE;
    uint32_t* Ln = lds + ((st + 1) & 1) * STAGE;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      Frags8<AW> f;
#pragma unroll
      for (int q = 0; q < AW; ++q)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          f.a[q][rb] = *reinterpret_cast<const uint4*>(L + q * WD + lane_off(s * 2 + h, wm * 64 + rb * 32 + l32));
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          f.b[q][cb] =
              *reinterpret_cast<const uint4*>(L + (AW + 2 * half + q) * WD + lane_off(s * 2 + h, c0 + cb * 32 + l32));
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          cr[rb][cb] = mma(f.a[0][rb], f.b[0][cb], cr[rb][cb]);
          if constexpr (!REAL) ci[rb][cb] = mma(f.a[2][rb], f.b[0][cb], ci[rb][cb]);
          cr[rb][cb] = mma(f.a[0][rb], f.b[1][cb], cr[rb][cb]);
          if constexpr (!REAL) ci[rb][cb] = mma(f.a[2][rb], f.b[1][cb], ci[rb][cb]);
          cr[rb][cb] = mma(f.a[1][rb], f.b[0][cb], cr[rb][cb]);
          if constexpr (!REAL) ci[rb][cb] = mma(f.a[3][rb], f.b[0][cb], ci[rb][cb]);
        }
      // the staged next stage goes to the idle buffer, half per step; after
      // the second half the registers take the stage after next (past the
      // end: the final stage again, in bounds, into a buffer never read)
      stage_store8<AW>(r, Ln, s, tid);
      if (s == 1) stage_load8<AW>(r, Ap, B0, B1, b_step, min(st + 2, g.nst - 1), tid);
    }
    lds_barrier();
  }

  if constexpr (OUT == OUT_HERK) {
    // one 128 x 128 column half at a time: complex FP32 (128 KB) or, for
    // real operands, real FP32 (64 KB, inside the 96 KB of the real core)
    using ET = typename std::conditional<REAL, float, float2>::type;
    ET* E = reinterpret_cast<ET*>(lds);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (half == c) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
              if constexpr (REAL)
                E[row * 128 + c0 + cb * 32 + l32] = cr[rb][cb][v];
              else
                E[row * 128 + c0 + cb * 32 + l32] = make_float2(cr[rb][cb][v], ci[rb][cb][v]);
            }
      }
      __syncthreads();
      double2* Pj = g.P + (size_t)jw * g.N * g.N;
#pragma unroll 4
      for (int e = tid; e < 128 * 128; e += GT8) {
        const int gi = ti * TM + (e >> 7), gj = tj * TN + c * 128 + (e & 127);
        if (gi < g.N && gj <= gi) {
          double2* p = Pj + (size_t)gi * g.N + gj;
          double2 y = *p;
          if constexpr (REAL) {
            y.x -= (double)E[e];
          } else {
            const float2 x = E[e];
            y.x -= (double)x.x;
            y.y -= (double)x.y;
          }
          *p = y;
        }
      }
      __syncthreads();
    }
    return;
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * 64 + cb * 32 + l32;
        const float re = cr[rb][cb][v], im = REAL ? 0.f : ci[rb][cb][v];
        if constexpr (OUT == OUT_TILED) {
          const int t = tj * TN + col;
          if constexpr (REAL) {
            // real M for the accumulation operands: [nI][T/32][4][TR][8] floats
            const size_t bs = (size_t)ti * g.nst_out + t / (2 * TK);
            const int kk = t % (2 * TK);
            reinterpret_cast<float*>(g.M)[((bs * 4 + (kk >> 3)) * TR + row) * 8 + (kk & 7)] = re;
          } else {
            const size_t bs = (size_t)ti * g.nst_out + t / TK;
            const int kk = t % TK;
            g.M[(bs * 4 + (kk >> 2)) * TR * 4 + row * 4 + (kk & 3)] = make_float2(re, im);
          }
        } else {
          const int gi = ti * TM + row, gt = tj * TN + col;
          if (gi < g.N && gt < g.T) g.M[(size_t)gi * g.ldm + gt] = make_float2(re, im);
        }
      }
}

template <int AW>
__device__ __forceinline__ void pp_frags(Frags8<AW>& f, const uint32_t* L, int s, int h, int wm, int half, int c0,
                                         int l32) {
#pragma unroll
  for (int q = 0; q < AW; ++q)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
      f.a[q][rb] = *reinterpret_cast<const uint4*>(L + q * WD + lane_off(s * 2 + h, wm * 64 + rb * 32 + l32));
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
      f.b[q][cb] =
          *reinterpret_cast<const uint4*>(L + (AW + 2 * half + q) * WD + lane_off(s * 2 + h, c0 + cb * 32 + l32));
}

// Workgroup barrier that no instruction is scheduled across (MFMAs included),
// so that each phase holds exactly its own work.
__device__ __forceinline__ void pp_barrier() {
  __builtin_amdgcn_sched_barrier(0);
  lds_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ void pp_mma(const Frags8<4>& f, floatx16 (&cr)[2][2], floatx16 (&ci)[2][2]) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      cr[rb][cb] = mma(f.a[0][rb], f.b[0][cb], cr[rb][cb]);
      ci[rb][cb] = mma(f.a[2][rb], f.b[0][cb], ci[rb][cb]);
      cr[rb][cb] = mma(f.a[0][rb], f.b[1][cb], cr[rb][cb]);
      ci[rb][cb] = mma(f.a[2][rb], f.b[1][cb], ci[rb][cb]);
      cr[rb][cb] = mma(f.a[1][rb], f.b[0][cb], cr[rb][cb]);
      ci[rb][cb] = mma(f.a[3][rb], f.b[0][cb], ci[rb][cb]);
    }
}

// ------------------------------------------- 8-wave ping-pong variant
// Same tile, operands and epilogues as gemm8_bf16x3_kernel; the two waves on
// each SIMD (group 0: waves 0-3, rows 0-63; group 1: waves 4-7, rows 64-127)
// alternate: while one group issues the MFMAs of a step from fragments it
// already holds, the other reads its next fragments from LDS and does the
// staging (its half of the next stage's LDS stores and global loads), and a
// workgroup barrier separates the phases.  Group 1 runs one phase behind.
template <int OUT>
__global__ __launch_bounds__(GT8, 1) void gemm8pp_bf16x3_kernel(GemmArgs g) {
  constexpr int AW = 4;
  constexpr int STAGE = (AW + 4) * WD;
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  int ti, tj, jw;
  decode_tile<OUT>(g, ti, tj, jw);
  const uint32_t* Ap = g.A + jw * g.omega_stride + ti * g.a_bstride;
  const uint32_t* B0 = g.B + jw * g.omega_stride + (size_t)(2 * tj) * g.b_bstride;
  const uint32_t* B1 = B0 + g.b_bstride;
  const size_t b_step = (size_t)g.b_words * WD;

  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = w >> 2, wn = w & 3;
  const int grp = wm;                              // wave-uniform
  const int half = wn >> 1, c0 = (wn & 1) * 64;
  const int l32 = lane & 31, h = lane >> 5;

  floatx16 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        cr[a][b][v] = 0.f;
        ci[a][b][v] = 0.f;
      }

  Staged8<AW> r;
  stage_load8<AW>(r, Ap, B0, B1, b_step, 0, tid);
  stage_store8<AW>(r, lds, 0, tid);
  stage_store8<AW>(r, lds, 1, tid);
  stage_load8<AW>(r, Ap, B0, B1, b_step, min(1, g.nst - 1), tid);
  lds_barrier();

  Frags8<AW> f;
  // Phases are separated by workgroup barriers; group 0 runs
  //   [fragments s=0 + staging] [MFMA] [fragments s=1] [MFMA]   per stage,
  // group 1 the same sequence one phase later (one extra barrier in front for
  // group 1, at the end for group 0), so every phase pairs one group's memory
  // work with the other's MFMAs.  Buffer (st+1)%2 is written in the phases
  // 4st and 4st+1 and read from 4st+4 on; its previous contents were last read
  // in phase 4st-1.
  if (grp == 1) pp_barrier();
  for (int st = 0; st < g.nst; ++st) {
    const uint32_t* L = lds + (st & 1) * STAGE;
    uint32_t* Ln = lds + ((st + 1) & 1) * STAGE;
    pp_frags<AW>(f, L, 0, h, wm, half, c0, l32);
    stage_store8<AW>(r, Ln, 0, tid);
    stage_store8<AW>(r, Ln, 1, tid);
    stage_load8<AW>(r, Ap, B0, B1, b_step, min(st + 2, g.nst - 1), tid);
    pp_barrier();
    pp_mma(f, cr, ci);
    pp_barrier();
    pp_frags<AW>(f, L, 1, h, wm, half, c0, l32);
    pp_barrier();
    pp_mma(f, cr, ci);
    pp_barrier();
  }
  if (grp == 0) pp_barrier();

  if constexpr (OUT == OUT_HERK) {
    float2* E = reinterpret_cast<float2*>(lds);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (half == c) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
              E[row * 128 + c0 + cb * 32 + l32] = make_float2(cr[rb][cb][v], ci[rb][cb][v]);
            }
      }
      __syncthreads();
      double2* Pj = g.P + (size_t)jw * g.N * g.N;
#pragma unroll 4
      for (int e = tid; e < 128 * 128; e += GT8) {
        const int gi = ti * TM + (e >> 7), gj = tj * TN + c * 128 + (e & 127);
        if (gi < g.N && gj <= gi) {
          const float2 x = E[e];
          double2* pp = Pj + (size_t)gi * g.N + gj;
          double2 y = *pp;
          y.x -= (double)x.x;
          y.y -= (double)x.y;
          *pp = y;
        }
      }
      __syncthreads();
    }
    return;
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * 64 + cb * 32 + l32;
        const float re = cr[rb][cb][v], im = ci[rb][cb][v];
        if constexpr (OUT == OUT_TILED) {
          const int t = tj * TN + col;
          const size_t bs = (size_t)ti * g.nst_out + t / TK;
          const int kk = t % TK;
          g.M[(bs * 4 + (kk >> 2)) * TR * 4 + row * 4 + (kk & 3)] = make_float2(re, im);
        } else {
          const int gi = ti * TM + row, gt = tj * TN + col;
          if (gi < g.N && gt < g.T) g.M[(size_t)gi * g.ldm + gt] = make_float2(re, im);
        }
      }
}

// ------------------------------------- three-multiplication core (Gauss form)
// Tile 128 x 256, 8 waves of 64 x 64 outputs, K stage = 16 complex k.  Each
// stage holds, per operand row, the hi and lo plane words of three real
// planes (A: 24 KB, B: two 128-column halves of 24 KB), copied straight from
// the tiled arrays into LDS (global_load_lds, no staging registers: the
// 192 accumulators of T1, T2, T3 leave no room for them), double-buffered
// (144 KB).  Per stage and wave: for each plane, 4 A and 4 B fragments and 12
// MFMAs (hi hi, hi lo, lo hi) -- 36 MFMAs and 24 LDS reads for 16 complex k,
// against 48 MFMAs and 24 reads in the four-product core.
//
// The two stage buffers are two distinct LDS arrays and the stage loop is
// unrolled by two, so that every buffer address is known at compile time.
// The compiler then sees that the fragment reads of one buffer do not alias
// the copy landing in the other, and lets the reads start while that copy is
// in flight; with one array indexed by the stage parity it has to wait for
// the copy (vmcnt 0) before the first read of every stage, which exposes the
// full load latency once per stage.
constexpr int ST3 = 18 * HWD;  // dwords per LDS stage (72 KB)

// DMA of stage st into LDS buffer L: 72 chunks of 1 KB (A plane words 0..5,
// then the two B halves' plane words), chunk q by wave q % 8.
__device__ __forceinline__ void stage_dma3(uint32_t* L, const GemmArgs& g, const uint32_t* Ap, const uint32_t* B0,
                                           const uint32_t* B1, int st, int w, int lane) {
  const size_t a_step = (size_t)g.a_words3 * HWD, b_step = (size_t)g.b_words3 * HWD;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int q = w + 8 * i;                 // wave-uniform
    const int region = q / 24, r = q % 24, pw = r >> 2, sub = r & 3;
    const uint32_t* src;
    if (region == 0) {
      src = Ap + (size_t)st * a_step + (size_t)pw * HWD;
    } else {
      const uint32_t* Bb = region == 1 ? B0 : B1;
      const int plane = pw < 4 ? pw : g.b_sum3 + (pw - 4);
      src = Bb + (size_t)st * b_step + (size_t)plane * HWD;
    }
    __builtin_amdgcn_global_load_lds(src + sub * 256 + lane * 4, (lds_void*)(L + q * 256), 16, 0, 0);
  }
}

template <int W>
__device__ inline floatx16 mma3(uint4 a, uint4 b, floatx16 c) {
  if constexpr (W == 0)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a), __builtin_bit_cast(halfx8, b), c, 0,
                                                  0, 0);
}

// The 12 MFMAs of one plane: A plane words at A (hi) and A + HWD (lo), B
// plane words at B and B + HWD, both already offset to this lane's rows.
template <int W>
__device__ __forceinline__ void plane_mma3(const uint32_t* A, const uint32_t* B, floatx16 (&t)[2][2]) {
  uint4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    ah[rb] = *reinterpret_cast<const uint4*>(A + rb * 128);
    al[rb] = *reinterpret_cast<const uint4*>(A + HWD + rb * 128);
  }
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    bh[cb] = *reinterpret_cast<const uint4*>(B + cb * 128);
    bl[cb] = *reinterpret_cast<const uint4*>(B + HWD + cb * 128);
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      t[rb][cb] = mma3<W>(ah[rb], bh[cb], t[rb][cb]);
      t[rb][cb] = mma3<W>(ah[rb], bl[cb], t[rb][cb]);
      t[rb][cb] = mma3<W>(al[rb], bh[cb], t[rb][cb]);
    }
}

// The 36 MFMAs of one stage from stage buffer L (A plane words 0..5, then the
// B halves' plane words from 6 and 12).
template <int W>
__device__ __forceinline__ void stage_mma3(const uint32_t* L, int aoff, int boff, floatx16 (&t)[3][2][2]) {
#pragma unroll
  for (int p = 0; p < 3; ++p) plane_mma3<W>(L + (2 * p) * HWD + aoff, L + boff + (2 * p) * HWD, t[p]);
}

// Combination of T1, T2, T3 into the complex result and the store: the
// projection's tiled or row-major M, or the lower-triangle update of P for
// the accumulation, either staged through LDS one 128 x 128 column half at a
// time (erow(r) points at staging row r, 128 float2) or, with erow null,
// read-modified-written by each lane from its registers (32 consecutive
// columns of one row per half wave).
//
// REAL: real operands, the sum over k in t[0] alone; the result is that sum
// (imaginary part zero), and the projection writes the real M layout the
// real accumulation operands are made from ([nI][T/32][4][TR][8] floats).
template <int OUT, int W, bool REAL = false, class ERow>
__device__ __forceinline__ void epilogue3(const GemmArgs& g, const floatx16 (&t)[3][2][2], int ti, int tj, int jw,
                                          int tid, ERow erow) {
  const int lane = tid & 63, w = tid >> 6;
  const int wm = w >> 2, wn = w & 3;
  const int half = wn >> 1, c0 = (wn & 1) * 64;
  const int l32 = lane & 31, h = lane >> 5;
  const float sg = g.sigma3;
  static_assert(!REAL || (W == 0 && std::is_same<ERow, std::nullptr_t>::value), "real operands: BF16, direct epilogue");
  if constexpr (OUT == OUT_HERK && std::is_same<ERow, std::nullptr_t>::value) {
    double2* Pj = g.P + (size_t)jw * g.N * g.N;
    const float* sj = W == 1 ? g.sa + (size_t)jw * g.s_stride : nullptr;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
          const int col = wn * 64 + cb * 32 + l32;
          const int gi = ti * TM + row, gj = tj * TN + col;
          if (gi < g.N && gj <= gi) {
            double2* pp = Pj + (size_t)gi * g.N + gj;
            double2 y = *pp;
            if constexpr (REAL) {
              y.x -= (double)t[0][rb][cb][v];
            } else {
              const float t1 = t[0][rb][cb][v], t2 = t[1][rb][cb][v], t3 = t[2][rb][cb][v];
              float un = 1.f;
              if constexpr (W == 1) un = 1.f / (sj[gi] * sj[gj]);
              y.x -= (double)((t1 + sg * t2) * un);
              y.y -= (double)((t3 - t1 + sg * t2) * un);
            }
            *pp = y;
          }
        }
    return;
  } else if constexpr (OUT == OUT_HERK) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (half == c) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
              const float t1 = t[0][rb][cb][v], t2 = t[1][rb][cb][v], t3 = t[2][rb][cb][v];
              float un = 1.f;
              if constexpr (W == 1) {
                const float* sj = g.sa + (size_t)jw * g.s_stride;
                un = 1.f / (sj[ti * TM + row] * sj[tj * TN + c * 128 + c0 + cb * 32 + l32]);
              }
              erow(row)[c0 + cb * 32 + l32] = make_float2((t1 + sg * t2) * un, (t3 - t1 + sg * t2) * un);
            }
      }
      __syncthreads();
      double2* Pj = g.P + (size_t)jw * g.N * g.N;
#pragma unroll 4
      for (int e = tid; e < 128 * 128; e += GT8) {
        const int gi = ti * TM + (e >> 7), gj = tj * TN + c * 128 + (e & 127);
        if (gi < g.N && gj <= gi) {
          const float2 x = erow(e >> 7)[e & 127];
          double2* pp = Pj + (size_t)gi * g.N + gj;
          double2 y = *pp;
          y.x -= (double)x.x;
          y.y -= (double)x.y;
          *pp = y;
        }
      }
      __syncthreads();
    }
    return;
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * 64 + cb * 32 + l32;
        float re, im;
        if constexpr (REAL) {
          re = t[0][rb][cb][v];
          im = 0.f;
        } else {
          const float t1 = t[0][rb][cb][v], t2 = t[1][rb][cb][v], t3 = t[2][rb][cb][v];
          float un = 1.f;
          if constexpr (W == 1) un = 1.f / (g.sa[ti * TM + row] * g.sb[tj * TN + col]);
          re = (t1 + sg * t2) * un;
          im = (t3 - t1 + sg * t2) * un;
        }
        if constexpr (OUT == OUT_TILED && REAL) {
          const int tt = tj * TN + col;
          const size_t bs = (size_t)ti * g.nst_out + tt / (2 * TK);
          const int kk = tt % (2 * TK);
          reinterpret_cast<float*>(g.M)[((bs * 4 + (kk >> 3)) * TR + row) * 8 + (kk & 7)] = re;
        } else if constexpr (OUT == OUT_TILED) {
          const int tt = tj * TN + col;
          const size_t bs = (size_t)ti * g.nst_out + tt / TK;
          const int kk = tt % TK;
          g.M[(bs * 4 + (kk >> 2)) * TR * 4 + row * 4 + (kk & 3)] = make_float2(re, im);
        } else {
          const int gi = ti * TM + row, gt = tj * TN + col;
          if (gi < g.N && gt < g.T) g.M[(size_t)gi * g.ldm + gt] = make_float2(re, im);
        }
      }
}

__device__ __forceinline__ void zero_acc3(floatx16 (&t)[3][2][2]) {
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) t[p][a][b][v] = 0.f;
}

// Two stage buffers of 72 KB: stage st + 1 is copied while stage st is
// multiplied.
template <int OUT, int W>
__global__ __launch_bounds__(GT8, 1) void gemm3m_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint32_t lds0[ST3];
  __shared__ __attribute__((aligned(16))) uint32_t lds1[ST3];
  int ti, tj, jw;
  decode_tile<OUT>(g, ti, tj, jw);
  const uint32_t* Ap = g.A + jw * g.omega_stride + ti * g.a_bstride;
  const uint32_t* B0 = g.B + jw * g.omega_stride + (size_t)(2 * tj) * g.b_bstride;
  const uint32_t* B1 = B0 + g.b_bstride;

  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = w >> 2, wn = w & 3;
  const int half = wn >> 1, c0 = (wn & 1) * 64;
  const int l32 = lane & 31, h = lane >> 5;

  floatx16 t[3][2][2];
  zero_acc3(t);
  const int aoff = lane_off3(h, wm * 64 + l32);
  const int boff = (6 + 6 * half) * HWD + lane_off3(h, c0 + l32);
  stage_dma3(lds0, g, Ap, B0, B1, 0, w, lane);
  for (int st = 0; st < g.nst; st += 2) {
    wait_vm0();
    lds_barrier();
    if (st + 1 < g.nst) stage_dma3(lds1, g, Ap, B0, B1, st + 1, w, lane);
    stage_mma3<W>(lds0, aoff, boff, t);
    if (st + 1 < g.nst) {
      wait_vm0();
      lds_barrier();
      if (st + 2 < g.nst) stage_dma3(lds0, g, Ap, B0, B1, st + 2, w, lane);
      stage_mma3<W>(lds1, aoff, boff, t);
    }
  }
  __syncthreads();   // every wave is done with the last stage's LDS

  // staging rows 0..63 in the first stage buffer, 64..127 in the second
  float2* E0 = reinterpret_cast<float2*>(lds0);
  float2* E1 = reinterpret_cast<float2*>(lds1);
  epilogue3<OUT, W>(g, t, ti, tj, jw, tid, [&](int r) { return r < 64 ? E0 + r * 128 : E1 + (r - 64) * 128; });
}

// ------------------------------------------------ six-slot ring of the core
// The same tile, operands and epilogue with finer staging: the LDS holds six
// plane slots of 24 KB (one plane's hi and lo words of A and of both B
// halves), and plane step i (stage i / 3, plane i % 3) is copied LEAD plane
// steps before it is multiplied (at most five: the slot it lands in was read
// at step i + LEAD - 6, before this step's barrier), against three in the
// two-buffer form, at one barrier per plane step instead of one per stage.
// Every plane step issues exactly three copies per wave (past the last step:
// the last step's source again, into a slot that is not read any more), so
// the copy of step i is complete once at most 3 (LEAD - 1) copies of this
// wave are outstanding.
constexpr int SL3 = 6 * HWD;  // dwords per plane slot (24 KB)

// Copy of plane p of stage st into slot S: chunk w of each of the slot's
// three regions (A, first B half, second B half), i.e. the hi (w < 4) or lo
// word of the plane, quarter w & 3.  Complex planes: words 2p (hi), 2p + 1
// (lo) of a stage of six (the B side's third plane from b_sum3 on).  REAL: a
// stage is one real block-stage of 32 k, planes p = 0, 1 its two halves of
// 16 k; hi words at p, lo words at 2 + p (four words per stage).
template <bool REAL>
__device__ __forceinline__ void slot_dma3(uint32_t* S, const GemmArgs& g, const uint32_t* Ap, const uint32_t* B0,
                                          const uint32_t* B1, int st, int p, int w, int lane) {
  const size_t a_step = (size_t)g.a_words3 * HWD, b_step = (size_t)g.b_words3 * HWD;
  const int hl = w >> 2, q = (w & 3) * 256 + lane * 4;
  const int pw = REAL ? p + 2 * hl : 2 * p + hl;
  const int bplane = (REAL || pw < 4) ? pw : g.b_sum3 + (pw - 4);
  const size_t bo = (size_t)st * b_step + (size_t)bplane * HWD + q;
  __builtin_amdgcn_global_load_lds(Ap + (size_t)st * a_step + (size_t)pw * HWD + q, (lds_void*)(S + w * 256), 16, 0,
                                   0);
  __builtin_amdgcn_global_load_lds(B0 + bo, (lds_void*)(S + 2 * HWD + w * 256), 16, 0, 0);
  __builtin_amdgcn_global_load_lds(B1 + bo, (lds_void*)(S + 4 * HWD + w * 256), 16, 0, 0);
}

// s_waitcnt vmcnt(N), N < 16 (expcnt and lgkmcnt left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt immediate");
  __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}

// Workgroup barrier between plane steps.  The acquire fences keep this wave's
// reads of the previous step above the barrier and the next copy below it; a
// release fence is not needed (the only LDS writes are the copies, waited for
// explicitly) and would make the compiler wait for every copy in flight.
__device__ __forceinline__ void ring_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int OUT, int W, int LEAD, bool REAL = false>
__global__ __launch_bounds__(GT8, 1) void gemm3r_kernel(GemmArgs g) {
  static_assert(LEAD >= 3 && LEAD <= 5, "slot (i + LEAD) % 6 must be free at plane step i");
  constexpr int NP = REAL ? 2 : 3;   // planes per stage
  __shared__ __attribute__((aligned(16))) uint32_t s0[SL3];
  __shared__ __attribute__((aligned(16))) uint32_t s1[SL3];
  __shared__ __attribute__((aligned(16))) uint32_t s2[SL3];
  __shared__ __attribute__((aligned(16))) uint32_t s3[SL3];
  __shared__ __attribute__((aligned(16))) uint32_t s4[SL3];
  __shared__ __attribute__((aligned(16))) uint32_t s5[SL3];
  uint32_t* const Q[6] = {s0, s1, s2, s3, s4, s5};
  int ti, tj, jw;
  decode_tile<OUT>(g, ti, tj, jw);
  const uint32_t* Ap = g.A + jw * g.omega_stride + ti * g.a_bstride;
  const uint32_t* B0 = g.B + jw * g.omega_stride + (size_t)(2 * tj) * g.b_bstride;
  const uint32_t* B1 = B0 + g.b_bstride;

  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = w >> 2, wn = w & 3;
  const int half = wn >> 1, c0 = (wn & 1) * 64;
  const int l32 = lane & 31, h = lane >> 5;

  floatx16 t[3][2][2];
  zero_acc3(t);
  const int aoff = lane_off3(h, wm * 64 + l32);
  const int boff = (2 + 2 * half) * HWD + lane_off3(h, c0 + l32);
  const int steps = NP * g.nst;
  auto issue = [&](int j, uint32_t* S) {
    j = min(j, steps - 1);
    slot_dma3<REAL>(S, g, Ap, B0, B1, j / NP, j % NP, w, lane);
  };
  // accumulator set of the plane at position k of a six-step group (real:
  // one set, in k order)
  auto acc = [&](int k) -> floatx16 (&)[2][2] { return t[REAL ? 0 : k % 3]; };
#pragma unroll
  for (int k = 0; k < LEAD; ++k) issue(k, Q[k]);
  int i = 0;
  for (; i + 6 <= steps; i += 6) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      wait_vm<3 * (LEAD - 1)>();
      ring_barrier();
      issue(i + k + LEAD, Q[(k + LEAD) % 6]);
      plane_mma3<W>(Q[k] + aoff, Q[k] + boff, acc(k));
    }
  }
  if (i < steps) {   // a multiple of NP steps is left: one stage (complex) or 1-2 stages (real)
#pragma unroll
    for (int k = 0; k < 6 - NP; ++k) {
      if (k < NP || i + k < steps) {
        wait_vm<3 * (LEAD - 1)>();
        ring_barrier();
        issue(i + k + LEAD, Q[(k + LEAD) % 6]);
        plane_mma3<W>(Q[k] + aoff, Q[k] + boff, acc(k));
      }
    }
  }
  wait_vm0();        // no copy into LDS outstanding at exit

  epilogue3<OUT, W, REAL>(g, t, ti, tj, jw, tid, nullptr);
}

template <int OUT>
int launch_gemm8pp(hipStream_t s, const GemmArgs& a, int grid, const char* name) {
  static int attr = 0;
  constexpr size_t lds_bytes = gemm8_lds_bytes<false>();
  if (!attr) {
    GW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm8pp_bf16x3_kernel<OUT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    attr = 1;
  }
  ProfScope prof(s, name);
  hipLaunchKernelGGL((gemm8pp_bf16x3_kernel<OUT>), dim3(grid), dim3(GT8), lds_bytes, s, a);
  GW_LAUNCHED("gemm8pp_bf16x3_kernel");
  return GW_OK;
}

template <int OUT, int DMA>
int enable_gemm_lds() {
  static int done = 0;
  if (done) return GW_OK;
  GW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_bf16x3_kernel<OUT, DMA>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmLds));
  done = 1;
  return GW_OK;
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
inline unsigned stream_blocks(size_t work) { return (unsigned)std::max<size_t>(1, std::min<size_t>((work + 255) / 256, 65536)); }

int count_lower_tiles(int nI) {
  int n = 0;
  for (int ti = 0; ti < nI; ++ti) n += ti / 2 + 1;
  return n;
}

// Sizes of one call's arrays (elements).
struct TiledDims {
  int nI, nIe, nstR, Tp, nT, nstT;
  size_t u_words, q_words, m_c64, x_words, sw_f32;
  size_t u3_words, q3_words, x3_words;   // the three-multiplication core's plane words
  size_t n_scale;                         // FP16 scales: U rows, pairs, M row maxima, X rows
  TiledDims(int N, int R, int T, int n_omega) {
    nI = cdiv(N, TR);
    nIe = (nI + 1) & ~1;
    nstR = cdiv(R, TK);
    Tp = cdiv(T, TN) * TN;
    nT = Tp / TR;
    nstT = Tp / TK;
    u_words = (size_t)nI * nstR * 4 * WD;
    q_words = (size_t)nT * nstR * 2 * WD;
    m_c64 = (size_t)nI * nstT * WD;
    x_words = (size_t)n_omega * nIe * nstT * 4 * WD;
    sw_f32 = (size_t)n_omega * Tp;
    u3_words = (size_t)nI * nstR * 6 * HWD;
    q3_words = (size_t)nT * nstR * 6 * HWD;
    x3_words = (size_t)n_omega * nIe * nstT * 8 * HWD;
    n_scale = (size_t)nIe * TR * 2 + Tp + (size_t)n_omega * nIe * TR;
    // one workspace layout serves both cores (the larger of each array)
    u_words = std::max(u_words, u3_words);
    q_words = std::max(q_words, q3_words);
    x_words = std::max(x_words, x3_words);
  }
  size_t bytes() const {
    return align_up(u_words * 4) + align_up(q_words * 4) + align_up(m_c64 * 8) + align_up(x_words * 4) +
           align_up(sw_f32 * 4) + align_up(n_scale * 4) + 8 * 256;   // + alignment of the scale arrays
  }
};

int launch_tile_u(hipStream_t s, const TiledDims& d, int N, int R, const float2* U, uint32_t* Uw) {
  hipLaunchKernelGGL(tile_u_kernel, dim3(stream_blocks((size_t)d.nI * d.nstR * 4 * TR)), dim3(256), 0, s, N, R, d.nI,
                     d.nstR, U, Uw);
  GW_LAUNCHED("tile_u_kernel");
  return GW_OK;
}

int launch_pair_product(hipStream_t s, const TiledDims& d, int R, const float2* po, const float2* pu, int nu, long tb,
                        int T, uint32_t* Q) {
  ProfScope prof(s, "pair_product_kernel");
  hipLaunchKernelGGL(pair_product_kernel, dim3((d.nstR + 1) / 2, d.nT), dim3(256), 0, s, R, d.nstR, d.nT, po, pu, nu,
                     tb, T, Q);
  GW_LAUNCHED("pair_product_kernel");
  return GW_OK;
}

template <int OUT, int DMA>
int launch_gemm_as(hipStream_t s, const GemmArgs& a, int grid, const char* name) {
  int st = enable_gemm_lds<OUT, DMA>();
  if (st != GW_OK) return st;
  ProfScope prof(s, name);
  hipLaunchKernelGGL((gemm_bf16x3_kernel<OUT, DMA>), dim3(grid), dim3(GT), kGemmLds, s, a);
  GW_LAUNCHED("gemm_bf16x3_kernel");
  return GW_OK;
}

template <int OUT, bool REAL = false>
int launch_gemm8(hipStream_t s, const GemmArgs& a, int grid, const char* name) {
  static int attr = 0;
  constexpr size_t lds_bytes = gemm8_lds_bytes<REAL>();
  if (!attr) {
    GW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm8_bf16x3_kernel<OUT, REAL>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    attr = 1;
  }
  ProfScope prof(s, name);
  hipLaunchKernelGGL((gemm8_bf16x3_kernel<OUT, REAL>), dim3(grid), dim3(GT8), lds_bytes, s, a);
  GW_LAUNCHED("gemm8_bf16x3_kernel");
  return GW_OK;
}

template <int OUT, int W>
int launch_gemm3m(hipStream_t s, const GemmArgs& a, int grid, const char* name) {
  ProfScope prof(s, name);  // stage buffers and slots are static LDS
  if (g_gemm3m_pipeline == 6) {
    if (g_gemm3m_lead == 3)
      hipLaunchKernelGGL((gemm3r_kernel<OUT, W, 3>), dim3(grid), dim3(GT8), 0, s, a);
    else if (g_gemm3m_lead == 4)
      hipLaunchKernelGGL((gemm3r_kernel<OUT, W, 4>), dim3(grid), dim3(GT8), 0, s, a);
    else
      hipLaunchKernelGGL((gemm3r_kernel<OUT, W, 5>), dim3(grid), dim3(GT8), 0, s, a);
    GW_LAUNCHED("gemm3r_kernel");
    return GW_OK;
  }
  hipLaunchKernelGGL((gemm3m_kernel<OUT, W>), dim3(grid), dim3(GT8), 0, s, a);
  GW_LAUNCHED("gemm3m_kernel");
  return GW_OK;
}

// Six-slot core for real operands (inversion-symmetric inputs), BF16 words.
template <int OUT>
int launch_gemm3r_real(hipStream_t s, const GemmArgs& a, int grid, const char* name) {
  ProfScope prof(s, name);
  if (g_gemm3m_lead == 3)
    hipLaunchKernelGGL((gemm3r_kernel<OUT, 0, 3, true>), dim3(grid), dim3(GT8), 0, s, a);
  else if (g_gemm3m_lead == 4)
    hipLaunchKernelGGL((gemm3r_kernel<OUT, 0, 4, true>), dim3(grid), dim3(GT8), 0, s, a);
  else
    hipLaunchKernelGGL((gemm3r_kernel<OUT, 0, 5, true>), dim3(grid), dim3(GT8), 0, s, a);
  GW_LAUNCHED("gemm3r_kernel");
  return GW_OK;
}

template <int OUT>
int launch_gemm(hipStream_t s, const GemmArgs& a, int grid, const char* name) {
  if (g_gemm_staging == 4) return launch_gemm8pp<OUT>(s, a, grid, name);
  if (g_gemm_staging == 3) return launch_gemm8<OUT>(s, a, grid, name);
  return g_gemm_staging == 2 ? launch_gemm_as<OUT, 1>(s, a, grid, name) : launch_gemm_as<OUT, 0>(s, a, grid, name);
}

__global__ void fill_f32_kernel(float* __restrict__ p, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// FP16 row scales of U (rows past N: 1), then the plane words.
template <int W>
int launch_tile_u3(hipStream_t s, const TiledDims& d, int N, int R, const float2* U, float* su, uint32_t* Uw) {
  if constexpr (W == 1) {
    hipLaunchKernelGGL(rowscale_u_kernel, dim3(N), dim3(256), 0, s, R, U, su);
    GW_LAUNCHED("rowscale_u_kernel");
    const int pad = d.nIe * TR - N;
    if (pad > 0) {
      hipLaunchKernelGGL(fill_f32_kernel, dim3(cdiv(pad, 256)), dim3(256), 0, s, su + N, pad, 1.f);
      GW_LAUNCHED("fill_f32_kernel");
    }
  }
  hipLaunchKernelGGL(tile_u3_kernel<W>, dim3(stream_blocks((size_t)d.nI * d.nstR * 2 * TR)), dim3(256), 0, s, N, R,
                     d.nI, d.nstR, U, su, Uw);
  GW_LAUNCHED("tile_u3_kernel");
  return GW_OK;
}

template <int W>
int launch_pair_product3(hipStream_t s, const TiledDims& d, int R, const float2* po, const float2* pu, int nu, long tb,
                         int T, const float* bmo, const float* bmu, float* sF, uint32_t* Q) {
  ProfScope prof(s, "pair_product_kernel");
  hipLaunchKernelGGL(pair_product3_kernel<W>, dim3((d.nstR + 1) / 2, d.nT), dim3(256), 0, s, R, d.nstR, d.nT, po,
                     pu, nu, tb, T, bmo, bmu, sF, Q);
  GW_LAUNCHED("pair_product3_kernel");
  return GW_OK;
}

int launch_bandmax(hipStream_t s, int rows, int R, const float2* psi, float* bm) {
  if (rows < 1) return GW_OK;
  hipLaunchKernelGGL(bandmax_kernel, dim3(rows), dim3(256), 0, s, R, psi, bm);
  GW_LAUNCHED("bandmax_kernel");
  return GW_OK;
}

// Projection arguments of the three-multiplication core: A = U planes, B =
// product planes (re, im, re + im).
void set_projection3(GemmArgs& a, const TiledDims& d, const uint32_t* Uw, const uint32_t* Q, int N, int T) {
  a.A = Uw;
  a.B = Q;
  a.a_words3 = 6;
  a.b_words3 = 6;
  a.b_sum3 = 4;
  a.sigma3 = -1.f;
  a.nst = d.nstR;
  a.a_bstride = (size_t)d.nstR * 6 * HWD;
  a.b_bstride = (size_t)d.nstR * 6 * HWD;
  a.nI = d.nI;
  a.nTj = d.Tp / TN;
  a.N = N;
  a.T = T;
}

// The three-multiplication pipeline.  Carver cv continues after the main
// arrays: the FP16 scales and band maxima are taken from it.
template <int W>
int tiled_project3(hipStream_t s, const TiledDims& d, int N, int R, int n_occ, int n_unocc, const float2* U,
                   const float2* po, const float2* pu, float2* M, uint32_t* Uw, uint32_t* Q, Carver& cv) {
  const int T = n_occ * n_unocc;
  float* su = cv.take<float>((size_t)d.nIe * TR);
  float* sF = cv.take<float>(d.Tp);
  float* bmo = cv.take<float>(n_occ);
  float* bmu = cv.take<float>(n_unocc);
  int st;
  if (W == 1) {
    if ((st = launch_bandmax(s, n_occ, R, po, bmo)) != GW_OK) return st;
    if ((st = launch_bandmax(s, n_unocc, R, pu, bmu)) != GW_OK) return st;
  }
  if ((st = launch_tile_u3<W>(s, d, N, R, U, su, Uw)) != GW_OK) return st;
  if ((st = launch_pair_product3<W>(s, d, R, po, pu, n_unocc, 0, T, bmo, bmu, sF, Q)) != GW_OK) return st;
  GemmArgs a{};
  set_projection3(a, d, Uw, Q, N, T);
  a.M = M;
  a.ldm = T;
  a.sa = su;
  a.sb = sF;
  return launch_gemm3m<OUT_ROWS, W>(s, a, d.nI * a.nTj, W ? "project_rows_f16_kernel" : "project_rows_bf16_kernel");
}

template <int W>
int tiled_polarization3(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, const TiledDims& dm,
                        const OmegaList& om, uint32_t* Uw, uint32_t* Q, float2* Mt, uint32_t* X, float* sw,
                        Carver& cv) {
  const float2* psi = static_cast<const float2*>(d.psi);
  const int nb = d.n_occ + d.n_unocc;
  const int n_tiles = count_lower_tiles(dm.nI);
  const int srows = dm.nIe * TR;
  float* su = cv.take<float>(srows);
  float* sF = cv.take<float>(dm.Tp);
  float* mrow = cv.take<float>(srows);
  float* sX = cv.take<float>((size_t)d.n_omega * srows);
  float* bm = cv.take<float>((size_t)d.n_k * nb);
  int st;
  if (W == 1 && (st = launch_bandmax(s, d.n_k * nb, d.R, psi, bm)) != GW_OK) return st;
  if ((st = launch_tile_u3<W>(s, dm, d.N, d.R, static_cast<const float2*>(d.U), su, Uw)) != GW_OK) return st;
  for (const Chunk& c : chunks) {
    // the chunk arrays are sized for the longest chunk; a shorter one pads with zeros
    TiledDims cd(d.N, d.R, c.T, d.n_omega);
    const float2* po = psi + ((size_t)c.k * nb + c.n0) * d.R;
    const float2* pu = psi + ((size_t)c.kq * nb + d.n_occ + c.u0) * d.R;
    const float* bmo = bm + (size_t)c.k * nb + c.n0;
    const float* bmu = bm + (size_t)c.kq * nb + d.n_occ + c.u0;
    hipLaunchKernelGGL(weights_sqrt_kernel, dim3(cdiv(cd.Tp, 256)), dim3(256), 0, s, d.eps, nb, d.n_occ, c, om,
                       cd.Tp, sw);
    GW_LAUNCHED("weights_sqrt_kernel");
    if ((st = launch_pair_product3<W>(s, cd, d.R, po, pu, c.nu, c.tb, c.T, bmo, bmu, sF, Q)) != GW_OK) return st;
    GemmArgs a{};
    set_projection3(a, cd, Uw, Q, d.N, c.T);
    a.M = Mt;
    a.nst_out = cd.nstT;
    a.sa = su;
    a.sb = sF;
    if ((st = launch_gemm3m<OUT_TILED, W>(s, a, cd.nI * a.nTj, W ? "project_f16_kernel" : "project_bf16_kernel")) !=
        GW_OK)
      return st;
    if (W == 1) {
      hipLaunchKernelGGL(mrow_kernel, dim3(cd.nIe), dim3(256), 0, s, cd.nI, cd.nstT, Mt, mrow);
      GW_LAUNCHED("mrow_kernel");
      hipLaunchKernelGGL(xscale_kernel, dim3(d.n_omega), dim3(256), 0, s, srows, cd.Tp, sw, mrow, sX);
      GW_LAUNCHED("xscale_kernel");
    }
    {
      ProfScope prof(s, "scale_split_kernel");
      hipLaunchKernelGGL(scale_split3_kernel<W>, dim3(stream_blocks((size_t)cd.nIe * cd.nstT * 2 * TR)), dim3(256), 0,
                         s, cd.nI, cd.nIe, cd.nstT, cd.Tp, d.n_omega, Mt, sw, sX, X);
      GW_LAUNCHED("scale_split3_kernel");
    }
    GemmArgs b{};
    b.A = X;
    b.B = X;
    b.a_words3 = 8;
    b.b_words3 = 8;
    b.b_sum3 = 6;
    b.sigma3 = 1.f;
    b.nst = cd.nstT;
    b.a_bstride = (size_t)cd.nstT * 8 * HWD;
    b.b_bstride = (size_t)cd.nstT * 8 * HWD;
    b.omega_stride = (size_t)cd.nIe * cd.nstT * 8 * HWD;
    b.nI = cd.nI;
    b.n_tiles = n_tiles;
    b.N = d.N;
    b.P = reinterpret_cast<double2*>(d.P);
    b.sa = sX;
    b.sb = sX;
    b.s_stride = srows;
    if ((st = launch_gemm3m<OUT_HERK, W>(s, b, n_tiles * d.n_omega, W ? "herk_f16_kernel" : "herk_bf16_kernel")) !=
        GW_OK)
      return st;
  }
  return GW_OK;
}

}  // namespace

size_t tiled_pol_workspace(int N, int R, int tc, int n_omega, size_t psi_rows) {
  return TiledDims(N, R, tc, n_omega).bytes() + align_up(psi_rows * 4);
}

size_t tiled_project_workspace(int N, int R, int n_occ, int n_unocc) {
  return TiledDims(N, R, n_occ * n_unocc, 0).bytes() + 2 * align_up((size_t)std::max(n_occ, n_unocc) * 4);
}

int tiled_polarization_f16(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                           const OmegaList& om, void* ws) {
  TiledDims dm(d.N, d.R, tc, d.n_omega);
  Carver cv(ws);
  uint32_t* Uw = cv.take<uint32_t>(dm.u_words);
  uint32_t* Q = cv.take<uint32_t>(dm.q_words);
  float2* Mt = cv.take<float2>(dm.m_c64);
  uint32_t* X = cv.take<uint32_t>(dm.x_words);
  float* sw = cv.take<float>(dm.sw_f32);
  return tiled_polarization3<1>(s, d, chunks, dm, om, Uw, Q, Mt, X, sw, cv);
}

int tiled_project_f16(hipStream_t s, int N, int R, int n_occ, int n_unocc, const float2* U, const float2* po,
                      const float2* pu, float2* M, void* ws) {
  TiledDims d(N, R, n_occ * n_unocc, 0);
  Carver cv(ws);
  uint32_t* Uw = cv.take<uint32_t>(d.u_words);
  uint32_t* Q = cv.take<uint32_t>(d.q_words);
  return tiled_project3<1>(s, d, N, R, n_occ, n_unocc, U, po, pu, M, Uw, Q, cv);
}

int tiled_default_chunk_pairs(int N, int R, int n_omega) {
  // Whole 256-pair tiles.  The projection grid (row blocks x pair tiles)
  // should fill complete rounds of the 256 compute units; the accumulation
  // adds each chunk into the FP64 P once per frequency, so longer chunks
  // amortise that read-modify-write (at N = 6000 and 16 frequencies it is
  // 9.2 GB per chunk); the chunk's arrays (product planes, 12 bytes per
  // complex value, and the scaled copies per frequency) stay within 32 GB.
  const long rows = cdiv(N, TR);
  const long nIe = (rows + 1) & ~1L;
  const size_t per_tile = (size_t)TN * ((size_t)cdiv(R, TK) * TK * 12 + (size_t)n_omega * nIe * TR * 16);
  const long cap = std::max<long>(1, std::min<long>(64, (long)(((size_t)32 << 30) / per_tile)));
  long best_x = 1;
  double best = -1.0;
  for (long x = 1; x <= cap; ++x) {
    const long wg = rows * x;
    const double fill = (double)wg / (double)(((wg + 255) / 256) * 256);
    if (fill > best + 0.005 || (fill > best - 0.005 && x > best_x)) {
      best = std::max(best, fill);
      best_x = x;
    }
  }
  return (int)(best_x * TN);
}

int tiled_project(hipStream_t s, int N, int R, int n_occ, int n_unocc, const float2* U, const float2* po,
                  const float2* pu, float2* M, void* ws) {
  const int T = n_occ * n_unocc;
  TiledDims d(N, R, T, 0);
  Carver cv(ws);
  uint32_t* Uw = cv.take<uint32_t>(d.u_words);
  uint32_t* Q = cv.take<uint32_t>(d.q_words);
  int st;
  if (g_complex_product == 3) return tiled_project3<0>(s, d, N, R, n_occ, n_unocc, U, po, pu, M, Uw, Q, cv);
  if ((st = launch_tile_u(s, d, N, R, U, Uw)) != GW_OK) return st;
  if ((st = launch_pair_product(s, d, R, po, pu, n_unocc, 0, T, Q)) != GW_OK) return st;
  GemmArgs a{};
  a.A = Uw;
  a.B = Q;
  a.b_words = 2;
  a.nst = d.nstR;
  a.a_bstride = (size_t)d.nstR * 4 * WD;
  a.b_bstride = (size_t)d.nstR * 2 * WD;
  a.nI = d.nI;
  a.nTj = d.Tp / TN;
  a.N = N;
  a.T = T;
  a.M = M;
  a.ldm = T;
  return launch_gemm<OUT_ROWS>(s, a, d.nI * a.nTj, "project_rows_bf16_kernel");
}

int tiled_polarization(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                       const OmegaList& om, void* ws) {
  TiledDims dm(d.N, d.R, tc, d.n_omega);
  Carver cv(ws);
  uint32_t* Uw = cv.take<uint32_t>(dm.u_words);
  uint32_t* Q = cv.take<uint32_t>(dm.q_words);
  float2* Mt = cv.take<float2>(dm.m_c64);
  uint32_t* X = cv.take<uint32_t>(dm.x_words);
  float* sw = cv.take<float>(dm.sw_f32);
  const float2* psi = static_cast<const float2*>(d.psi);
  const int nb = d.n_occ + d.n_unocc;
  int st;
  const int n_tiles = count_lower_tiles(dm.nI);
  if (g_complex_product == 3) return tiled_polarization3<0>(s, d, chunks, dm, om, Uw, Q, Mt, X, sw, cv);
  if ((st = launch_tile_u(s, dm, d.N, d.R, static_cast<const float2*>(d.U), Uw)) != GW_OK) return st;
  for (const Chunk& c : chunks) {
    // the chunk arrays are sized for tc pairs; a shorter last chunk pads with zeros
    TiledDims cd(d.N, d.R, c.T, d.n_omega);
    const float2* po = psi + ((size_t)c.k * nb + c.n0) * d.R;
    const float2* pu = psi + ((size_t)c.kq * nb + d.n_occ + c.u0) * d.R;
    hipLaunchKernelGGL(weights_sqrt_kernel, dim3(cdiv(cd.Tp, 256)), dim3(256), 0, s, d.eps, nb, d.n_occ, c, om, cd.Tp,
                       sw);
    GW_LAUNCHED("weights_sqrt_kernel");
    if ((st = launch_pair_product(s, cd, d.R, po, pu, c.nu, c.tb, c.T, Q)) != GW_OK) return st;
    GemmArgs a{};
    a.A = Uw;
    a.B = Q;
    a.b_words = 2;
    a.nst = cd.nstR;
    a.a_bstride = (size_t)cd.nstR * 4 * WD;
    a.b_bstride = (size_t)cd.nstR * 2 * WD;
    a.nI = cd.nI;
    a.nTj = cd.Tp / TN;
    a.N = d.N;
    a.T = c.T;
    a.M = Mt;
    a.nst_out = cd.nstT;
    if ((st = launch_gemm<OUT_TILED>(s, a, cd.nI * a.nTj, "project_bf16_kernel")) != GW_OK) return st;
    {
      ProfScope prof(s, "scale_split_kernel");
      hipLaunchKernelGGL(scale_split_kernel, dim3(stream_blocks((size_t)cd.nIe * cd.nstT * 4 * TR)), dim3(256), 0, s,
                         cd.nI, cd.nIe, cd.nstT, cd.Tp, d.n_omega, Mt, sw, X);
      GW_LAUNCHED("scale_split_kernel");
    }
    GemmArgs b{};
    b.A = X;
    b.B = X;
    b.b_words = 4;
    b.nst = cd.nstT;
    b.a_bstride = (size_t)cd.nstT * 4 * WD;
    b.b_bstride = (size_t)cd.nstT * 4 * WD;
    b.omega_stride = (size_t)cd.nIe * cd.nstT * 4 * WD;
    b.nI = cd.nI;
    b.n_tiles = n_tiles;
    b.N = d.N;
    b.P = reinterpret_cast<double2*>(d.P);
    if ((st = launch_gemm<OUT_HERK>(s, b, n_tiles * d.n_omega, "herk_bf16_kernel")) != GW_OK) return st;
  }
  return GW_OK;
}

// ---------------------------------------------------------- real path
// Real U and wave functions (the inversion-symmetric case): P is real
// symmetric; every contraction runs on the real form of the GEMM core (a
// quarter of the complex path's MFMA work).
struct RealDims {
  int nI, nIe, nstR, Tp, nT, nstT;
  size_t u_words, q_words, m_f32, x_words, sw_f32;
  RealDims(int N, int R, int T, int n_omega) {
    nI = cdiv(N, TR);
    nIe = (nI + 1) & ~1;
    nstR = cdiv(R, 2 * TK);
    Tp = cdiv(T, TN) * TN;
    nT = Tp / TR;
    nstT = Tp / (2 * TK);
    u_words = (size_t)nI * nstR * 2 * WD;
    q_words = (size_t)nT * nstR * 2 * WD;
    m_f32 = (size_t)nI * nstT * 4 * TR * 8;
    x_words = (size_t)n_omega * nIe * nstT * 2 * WD;
    sw_f32 = (size_t)n_omega * Tp;
  }
  size_t bytes() const {
    return align_up(u_words * 4) + align_up(q_words * 4) + align_up(m_f32 * 4) + align_up(x_words * 4) +
           align_up(sw_f32 * 4);
  }
};

size_t tiled_pol_workspace_real(int N, int R, int tc, int n_omega) { return RealDims(N, R, tc, n_omega).bytes(); }

int tiled_polarization_real(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                            const OmegaList& om, void* ws) {
  RealDims dm(d.N, d.R, tc, d.n_omega);
  Carver cv(ws);
  uint32_t* Uw = cv.take<uint32_t>(dm.u_words);
  uint32_t* Q = cv.take<uint32_t>(dm.q_words);
  float* Mt = cv.take<float>(dm.m_f32);
  uint32_t* X = cv.take<uint32_t>(dm.x_words);
  float* sw = cv.take<float>(dm.sw_f32);
  const float* psi = static_cast<const float*>(d.psi);
  const int nb = d.n_occ + d.n_unocc;
  hipLaunchKernelGGL(tile_u_real_kernel, dim3(stream_blocks((size_t)dm.nI * dm.nstR * 4 * TR)), dim3(256), 0, s, d.N,
                     d.R, dm.nI, dm.nstR, static_cast<const float*>(d.U), Uw);
  GW_LAUNCHED("tile_u_real_kernel");
  const int n_tiles = count_lower_tiles(dm.nI);
  int st;
  for (const Chunk& c : chunks) {
    RealDims cd(d.N, d.R, c.T, d.n_omega);
    const float* po = psi + ((size_t)c.k * nb + c.n0) * d.R;
    const float* pu = psi + ((size_t)c.kq * nb + d.n_occ + c.u0) * d.R;
    hipLaunchKernelGGL(weights_sqrt_kernel, dim3(cdiv(cd.Tp, 256)), dim3(256), 0, s, d.eps, nb, d.n_occ, c, om, cd.Tp,
                       sw);
    GW_LAUNCHED("weights_sqrt_kernel");
    {
      ProfScope prof(s, "pair_product_kernel");
      hipLaunchKernelGGL(pair_product_real_kernel, dim3((cd.nstR + 1) / 2, cd.nT), dim3(256), 0, s, d.R, cd.nstR,
                         cd.nT, po, pu, c.nu, c.tb, c.T, Q);
      GW_LAUNCHED("pair_product_real_kernel");
    }
    GemmArgs a{};
    a.A = Uw;
    a.B = Q;
    a.b_words = 2;
    a.nst = cd.nstR;
    a.a_bstride = (size_t)cd.nstR * 2 * WD;
    a.b_bstride = (size_t)cd.nstR * 2 * WD;
    a.nI = cd.nI;
    a.nTj = cd.Tp / TN;
    a.N = d.N;
    a.T = c.T;
    a.M = reinterpret_cast<float2*>(Mt);
    a.nst_out = cd.nstT;
    a.a_words3 = a.b_words3 = 4;   // six-slot core: hi, hi, lo, lo plane words per real stage
    if ((st = g_real_core == 2 ? launch_gemm3r_real<OUT_TILED>(s, a, cd.nI * a.nTj, "project_bf16_kernel")
                               : launch_gemm8<OUT_TILED, true>(s, a, cd.nI * a.nTj, "project_bf16_kernel")) != GW_OK)
      return st;
    {
      ProfScope prof(s, "scale_split_kernel");
      hipLaunchKernelGGL(scale_split_real_kernel, dim3(stream_blocks((size_t)cd.nIe * cd.nstT * 4 * TR)), dim3(256), 0,
                         s, cd.nI, cd.nIe, cd.nstT, cd.Tp, d.n_omega, Mt, sw, X);
      GW_LAUNCHED("scale_split_real_kernel");
    }
    GemmArgs b{};
    b.A = X;
    b.B = X;
    b.b_words = 2;
    b.nst = cd.nstT;
    b.a_bstride = (size_t)cd.nstT * 2 * WD;
    b.b_bstride = (size_t)cd.nstT * 2 * WD;
    b.omega_stride = (size_t)cd.nIe * cd.nstT * 2 * WD;
    b.nI = cd.nI;
    b.n_tiles = n_tiles;
    b.N = d.N;
    b.P = reinterpret_cast<double2*>(d.P);
    b.a_words3 = b.b_words3 = 4;
    if ((st = g_real_core == 2 ? launch_gemm3r_real<OUT_HERK>(s, b, n_tiles * d.n_omega, "herk_bf16_kernel")
                               : launch_gemm8<OUT_HERK, true>(s, b, n_tiles * d.n_omega, "herk_bf16_kernel")) != GW_OK)
      return st;
  }
  return GW_OK;
}

// ------------------------------------------------ correlation self-energy
// Quadratic forms q_j[n'] = m^H (W_j - diag v) m of Eq. SEc_AC for one state
// and one transfer, split BF16 on the GEMM core: the projections m of the
// products conj(psi_state) psi_n' (all bands n'), then Y_j = W^c_j M and the
// column dots.
// Batched quadratic forms of the self-energy: the states of a batch share
// W^c(t), so their projections sit side by side as the columns of one operand,
// each state's bands padded to whole 256-column tiles.
struct SigmaDims {
  int nI, nstR, nstN, nbp, cols, nTb;
  size_t u_words, q_words, m_c64, mt_words, w_words, part;
  SigmaDims(int N, int R, int nb, int g) {
    nI = cdiv(N, TR);
    nstR = cdiv(R, TK);
    nstN = cdiv(N, TK);
    nbp = cdiv(nb, TN) * TN;
    cols = g * nbp;
    nTb = cols / TR;
    // word arrays sized for the larger of the two GEMM cores' layouts
    // (four-product: 8 / 4 HWD per block-stage for A / B; three-product: 6)
    u_words = (size_t)nI * nstR * 4 * WD;
    q_words = (size_t)(nbp / TR) * nstR * 6 * HWD;   // pair products of one state
    m_c64 = (size_t)N * cols;
    mt_words = (size_t)nTb * nstN * 6 * HWD;
    w_words = (size_t)nI * nstN * 4 * WD;
    part = (size_t)CD_CHUNKS * cols;
  }
  size_t bytes() const {
    return align_up(u_words * 4) + align_up(q_words * 4) + 2 * align_up(m_c64 * 8) + align_up(mt_words * 4) +
           align_up(w_words * 4) + align_up(part * 8);
  }
};

namespace {
__global__ void zero_u32_kernel(uint32_t* __restrict__ p, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) p[e] = 0u;
}
}  // namespace

int tiled_sigma_cols(int nb, int g) { return g * (cdiv(nb, TN) * TN); }

size_t tiled_sigma_workspace(int N, int R, int nb, int g) { return SigmaDims(N, R, nb, g).bytes(); }

int tiled_sigma_quadforms(hipStream_t s, int N, int R, int nb, int g, int n_mesh, const float2* U, bool tile_u,
                          const float2* const* psi_state, const float2* const* psi_all, const double2* W,
                          const double* v, double* q, void* ws) {
  SigmaDims d(N, R, nb, g);
  Carver cv(ws);
  uint32_t* Uw = cv.take<uint32_t>(d.u_words);
  uint32_t* Q = cv.take<uint32_t>(d.q_words);
  float2* M = cv.take<float2>(d.m_c64);
  float2* Y = cv.take<float2>(d.m_c64);
  uint32_t* Mt = cv.take<uint32_t>(d.mt_words);
  uint32_t* Ww = cv.take<uint32_t>(d.w_words);
  double* part = cv.take<double>(d.part);
  const int rows_per_chunk = cdiv(N, CD_CHUNKS);
  int st;
  TiledDims td(N, R, nb, 0);
  // the padding columns of every state's block stay zero
  hipLaunchKernelGGL(zero_u32_kernel, dim3(stream_blocks(d.m_c64 * 2)), dim3(256), 0, s,
                     reinterpret_cast<uint32_t*>(M), d.m_c64 * 2);
  GW_LAUNCHED("zero_u32_kernel");
  if (g_complex_product == 3) {
    // three-multiplication core: U and product planes (re, im, re + im), the
    // projections, then per frequency Y = W^c M on W^c and M planes
    if (tile_u && (st = launch_tile_u3<0>(s, td, N, R, U, nullptr, Uw)) != GW_OK) return st;
    for (int i = 0; i < g; ++i) {
      if ((st = launch_pair_product3<0>(s, td, R, psi_state[i], psi_all[i], nb, 0, nb, nullptr, nullptr, nullptr, Q)) !=
          GW_OK)
        return st;
      GemmArgs a{};
      set_projection3(a, td, Uw, Q, N, nb);
      a.M = M + (size_t)i * d.nbp;
      a.ldm = d.cols;
      if ((st = launch_gemm3m<OUT_ROWS, 0>(s, a, d.nI * a.nTj, "sigma_project_kernel")) != GW_OK) return st;
    }
    hipLaunchKernelGGL(tile_cols3_kernel, dim3(stream_blocks((size_t)d.nTb * d.nstN * 2 * TR)), dim3(256), 0, s, N,
                       d.cols, d.nTb, d.nstN, M, (long)d.cols, Mt);
    GW_LAUNCHED("tile_cols3_kernel");
    for (int j = 0; j < n_mesh; ++j) {
      hipLaunchKernelGGL(tile_wc3_kernel, dim3(stream_blocks((size_t)d.nI * d.nstN * 2 * TR)), dim3(256), 0, s, N,
                         d.nI, d.nstN, W + (size_t)j * N * N, v, Ww);
      GW_LAUNCHED("tile_wc3_kernel");
      GemmArgs b{};
      b.A = Ww;
      b.B = Mt;
      b.a_words3 = 6;
      b.b_words3 = 6;
      b.b_sum3 = 4;
      b.sigma3 = -1.f;
      b.nst = d.nstN;
      b.a_bstride = (size_t)d.nstN * 6 * HWD;
      b.b_bstride = (size_t)d.nstN * 6 * HWD;
      b.nI = d.nI;
      b.nTj = d.cols / TN;
      b.N = N;
      b.T = d.cols;
      b.M = Y;
      b.ldm = d.cols;
      if ((st = launch_gemm3m<OUT_ROWS, 0>(s, b, d.nI * b.nTj, "sigma_wm_kernel")) != GW_OK) return st;
      hipLaunchKernelGGL(coldot_f32_kernel, dim3(cdiv(d.cols, 32), CD_CHUNKS), dim3(256), 0, s, N, d.cols, M, Y,
                         (long)d.cols, rows_per_chunk, part);
      GW_LAUNCHED("coldot_f32_kernel");
      hipLaunchKernelGGL(coldot_reduce_kernel, dim3(cdiv(d.cols, 256)), dim3(256), 0, s, d.cols, CD_CHUNKS, part,
                         q + (size_t)j * d.cols);
      GW_LAUNCHED("coldot_reduce_kernel");
    }
    return GW_OK;
  }
  if (tile_u && (st = launch_tile_u(s, td, N, R, U, Uw)) != GW_OK) return st;
  for (int i = 0; i < g; ++i) {
    if ((st = launch_pair_product(s, td, R, psi_state[i], psi_all[i], nb, 0, nb, Q)) != GW_OK) return st;
    GemmArgs a{};
    a.A = Uw;
    a.B = Q;
    a.b_words = 2;
    a.nst = d.nstR;
    a.a_bstride = (size_t)d.nstR * 4 * WD;
    a.b_bstride = (size_t)d.nstR * 2 * WD;
    a.nI = d.nI;
    a.nTj = d.nbp / TN;
    a.N = N;
    a.T = nb;
    a.M = M + (size_t)i * d.nbp;
    a.ldm = d.cols;
    if ((st = launch_gemm<OUT_ROWS>(s, a, d.nI * a.nTj, "sigma_project_kernel")) != GW_OK) return st;
  }
  hipLaunchKernelGGL(tile_cols_kernel, dim3(stream_blocks((size_t)d.nTb * d.nstN * 4 * TR)), dim3(256), 0, s, N,
                     d.cols, d.nTb, d.nstN, M, (long)d.cols, Mt);
  GW_LAUNCHED("tile_cols_kernel");
  for (int j = 0; j < n_mesh; ++j) {
    hipLaunchKernelGGL(tile_wc_kernel, dim3(stream_blocks((size_t)d.nI * d.nstN * 4 * TR)), dim3(256), 0, s, N, d.nI,
                       d.nstN, W + (size_t)j * N * N, v, Ww);
    GW_LAUNCHED("tile_wc_kernel");
    GemmArgs b{};
    b.A = Ww;
    b.B = Mt;
    b.b_words = 2;
    b.nst = d.nstN;
    b.a_bstride = (size_t)d.nstN * 4 * WD;
    b.b_bstride = (size_t)d.nstN * 2 * WD;
    b.nI = d.nI;
    b.nTj = d.cols / TN;
    b.N = N;
    b.T = d.cols;
    b.M = Y;
    b.ldm = d.cols;
    if ((st = launch_gemm<OUT_ROWS>(s, b, d.nI * b.nTj, "sigma_wm_kernel")) != GW_OK) return st;
    hipLaunchKernelGGL(coldot_f32_kernel, dim3(cdiv(d.cols, 32), CD_CHUNKS), dim3(256), 0, s, N, d.cols, M, Y,
                       (long)d.cols, rows_per_chunk, part);
    GW_LAUNCHED("coldot_f32_kernel");
    hipLaunchKernelGGL(coldot_reduce_kernel, dim3(cdiv(d.cols, 256)), dim3(256), 0, s, d.cols, CD_CHUNKS, part,
                       q + (size_t)j * d.cols);
    GW_LAUNCHED("coldot_reduce_kernel");
  }
  return GW_OK;
}

}  // namespace gw
